// Small float64 kernels of one s-step block, each run by a single
// workgroup: partial Cholesky with incremental condition estimation
// (Alg. 3), the R-factor combination of BCGS2 (Alg. 4), Hessenberg
// recovery through the change-of-basis matrix followed by Givens rotations
// and the per-column convergence test, and the final back substitution.
// These are latency-bound (a few hundred sequential steps at most).
#include "internal.h"

namespace sgm {

namespace {

constexpr int kSmallBlock = 256;

__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += red[i];
  return t;
}

// Largest eigenvalue of [[a, b], [b, c]] and a unit eigenvector (u, v).
__device__ void top_eig_2x2(double a, double b, double c, double& lam,
                            double& u, double& v) {
  lam = 0.5 * (a + c) + hypot(0.5 * (a - c), b);
  if (b == 0.0) {
    if (a >= c) { u = 1.0; v = 0.0; } else { u = 0.0; v = 1.0; }
    return;
  }
  double x, y;
  if (a >= c) { x = lam - c; y = b; } else { x = b; y = lam - a; }
  const double nr = hypot(x, y);
  u = x / nr;
  v = y / nr;
}

// Partial Cholesky (Alg. 3) of the leading s x s block of G, right-looking
// in place in the upper triangle of a work copy (LDS when s <= 128).  After
// column j the incremental condition estimator updates its two approximate
// singular vectors: y for the largest singular value (|y^T R|) and
// d = R^{-T} x for the smallest (1/|d|), each through a 2x2 symmetric
// eigenproblem in (sin, cos); the factorisation stops before a column whose
// pivot is not positive and finite, or whose estimate exceeds omega.
// Outputs: p, R (p x p upper), Rinv = R^{-1} (explicit, by column-wise back
// substitution), both column-major with leading dimension ldr.
__global__ __launch_bounds__(kSmallBlock) void k_pchol(
    const double* __restrict__ G, int ldg, int smax, const int* s_dev,
    double omega, double* __restrict__ R, double* __restrict__ Rinv, int ldr,
    int* p_out, double* scratch) {
  __shared__ double As[kSmallLds * kSmallLds];
  __shared__ double ys[1024], ds[1024];
  __shared__ double red[kSmallBlock / kWave];
  __shared__ double bc[4];
  const int tid = threadIdx.x;
  int s = smax;
  if (s_dev) s = min(s, *s_dev);
  if (s > 1024) s = 1024;
  double* Aw = s <= kSmallLds ? As : scratch;
  const int la = s <= kSmallLds ? (s > 0 ? s : 1) : smax;
  for (int e = tid; e < s * s; e += kSmallBlock) {
    const int i = e % s, j = e / s;
    Aw[j * la + i] = G[(int64_t)j * ldg + i];
  }
  __syncthreads();
  double smax2 = 0.0, dn2 = 0.0;  // estimator state (uniform across threads)
  int p = s;
  for (int j = 0; j < s; ++j) {
    const double piv = Aw[j * la + j];
    if (!(piv > 0.0) || !isfinite(piv)) { p = j; break; }
    const double rjj = sqrt(piv);
    double kappa = 1.0;
    if (j == 0) {
      if (tid == 0) { ys[0] = 1.0; ds[0] = 1.0 / rjj; }
      smax2 = piv;
      dn2 = 1.0 / piv;
    } else {
      double a = 0.0, a2 = 0.0;
      for (int t = tid; t < j; t += kSmallBlock) {
        const double v = Aw[j * la + t];  // R(t, j)
        a += ys[t] * v;
        a2 += v * ds[t];
      }
      a = block_sum(a, red);
      a2 = block_sum(a2, red);
      double lam1, s1, c1, lam2, s2, c2;
      top_eig_2x2(smax2 + a * a, a * rjj, rjj * rjj, lam1, s1, c1);
      top_eig_2x2(dn2 + (a2 / rjj) * (a2 / rjj), -a2 / (rjj * rjj),
                  1.0 / (rjj * rjj), lam2, s2, c2);
      smax2 = lam1;
      dn2 = lam2;
      kappa = sqrt(smax2 * dn2);
      __syncthreads();
      for (int t = tid; t < j; t += kSmallBlock) {
        ys[t] *= s1;
        ds[t] *= s2;
      }
      if (tid == 0) {
        ys[j] = c1;
        ds[j] = (c2 - s2 * a2) / rjj;
      }
    }
    if (!(kappa <= omega)) { p = j; break; }
    __syncthreads();
    if (tid == 0) Aw[j * la + j] = rjj;
    for (int k = j + 1 + tid; k < s; k += kSmallBlock) Aw[k * la + j] /= rjj;
    __syncthreads();
    const int rem = s - j - 1;
    for (int e = tid; e < rem * rem; e += kSmallBlock) {
      const int kk = j + 1 + e % rem, ll = j + 1 + e / rem;
      if (kk <= ll) Aw[ll * la + kk] -= Aw[kk * la + j] * Aw[ll * la + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) *p_out = p;
  for (int e = tid; e < p * p; e += kSmallBlock) {
    const int i = e % p, j = e / p;
    R[(int64_t)j * ldr + i] = i <= j ? Aw[j * la + i] : 0.0;
  }
  __syncthreads();
  // Rinv column c by back substitution: R x = e_c.
  for (int c = tid; c < p; c += kSmallBlock) {
    double* xc = Rinv + (int64_t)c * ldr;
    for (int r = c + 1; r < p; ++r) xc[r] = 0.0;
    xc[c] = 1.0 / Aw[c * la + c];
    for (int r = c - 1; r >= 0; --r) {
      double acc = 0.0;
      for (int t = r + 1; t <= c; ++t) acc += Aw[t * la + r] * xc[t];
      xc[r] = -acc / Aw[r * la + r];
    }
  }
}

// Combine both BCGS passes (Alg. 4): R(1:i, k) = W(:, 1:p) + R2(:, 1:p) Z,
// R(k, k) = Zt Z, p = p2.  A breakdown (p2 = 0) yields the single column
// of the first new vector's coefficients with R(k, k) = 0.
__global__ __launch_bounds__(kSmallBlock) void k_combine(
    const double* __restrict__ W, int ldw, const double* __restrict__ R2,
    int ldr2, const double* __restrict__ Z, const double* __restrict__ Zt,
    int ldz, int i, int* ctrl, double* __restrict__ Rtop, int ldt,
    double* __restrict__ Rkk, int ldk) {
  const int p1 = ctrl[C_P1], p2 = ctrl[C_P2];
  const int tid = threadIdx.x;
  if (p2 > 0) {
    for (int e = tid; e < i * p2; e += kSmallBlock) {
      const int r = e % i, c = e / i;
      double acc = 0.0;
      for (int t = 0; t <= c; ++t)
        acc += R2[(int64_t)t * ldr2 + r] * Z[(int64_t)c * ldz + t];
      Rtop[(int64_t)c * ldt + r] = W[(int64_t)c * ldw + r] + acc;
    }
    for (int e = tid; e < p2 * p2; e += kSmallBlock) {
      const int r = e % p2, c = e / p2;
      double acc = 0.0;
      for (int t = r; t <= c; ++t)
        acc += Zt[(int64_t)t * ldz + r] * Z[(int64_t)c * ldz + t];
      Rkk[(int64_t)c * ldk + r] = r <= c ? acc : 0.0;
    }
    if (tid == 0) {
      ctrl[C_PH] = p2;
      ctrl[C_BREAK] = 0;
    }
  } else {
    for (int r = tid; r < i; r += kSmallBlock) {
      double v = W[r];
      if (p1 > 0) v += R2[r] * Z[0];
      Rtop[r] = v;
    }
    if (tid == 0) {
      Rkk[0] = 0.0;
      ctrl[C_PH] = 1;
      ctrl[C_BREAK] = 1;
    }
  }
}

// Hessenberg recovery for the block started at basis vector nb (1-based):
// with Rt = [e_nb | R(1:nb+p, k)] and B the (p+1) x p change-of-basis matrix
// of the recurrence records, H(1:nb+p, nb:nb+p-1) = (Rt B - [H(1:nb,
// 1:nb-1) X; 0]) T^{-1}, X = Rt(1:nb-1, 1:p), T = Rt(nb:nb+p-1, 1:p).
// Then the new columns get the earlier Givens rotations, new rotations are
// formed column by column, and the relative residual estimate
// |g(c+1)| / beta0 of every new column is written to res_out; the block
// stops at the first column that meets tol.
__global__ __launch_bounds__(kSmallBlock) void k_hess_givens(
    double* __restrict__ Hraw, double* __restrict__ Hr, int ldh,
    double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
    int nb, const double* __restrict__ Rtop, int ldt,
    const double* __restrict__ Rkk, int ldk, const double* __restrict__ rec,
    int n_rec, const double* __restrict__ beta0, double tol, int* ctrl,
    double* __restrict__ res_out) {
  const int p = ctrl[C_PH];
  const int tid = threadIdx.x;
  const int i0 = nb - 1;  // 0-based row of e_nb in Rt; first new column
  auto Rt = [&](int r, int c) -> double {  // (nb+p) x (p+1)
    if (c == 0) return r == i0 ? 1.0 : 0.0;
    if (r < nb) return Rtop[(int64_t)(c - 1) * ldt + r];
    return Rkk[(int64_t)(c - 1) * ldk + (r - nb)];
  };
  // Each thread owns rows of the new block of H; the row solve with T is
  // independent per row.
  for (int r = tid; r < nb + p; r += kSmallBlock) {
    double* hrow = Hraw + r;  // element (r, c) at hrow[c * ldh]
    for (int j = 0; j < p; ++j) {
      const int q = j % n_rec;
      const double th = rec[3 * q], ga = rec[3 * q + 1], de = rec[3 * q + 2];
      double m = th * Rt(r, j) + ga * Rt(r, j + 1);
      if (j >= 1) m += de * Rt(r, j - 1);
      if (r < nb && nb > 1) {
        double acc = 0.0;
        for (int t = 0; t < nb - 1; ++t)
          acc += Hraw[(int64_t)t * ldh + r] * Rt(t, j);
        m -= acc;
      }
      // forward substitution with T (T(a, b) = Rt(i0 + a, b))
      for (int t = 0; t < j; ++t) m -= hrow[(int64_t)(i0 + t) * ldh] * Rt(i0 + t, j);
      hrow[(int64_t)(i0 + j) * ldh] = m / Rt(i0 + j, j);
    }
  }
  __syncthreads();
  // Rotated copy of the new columns (rows 0..c+1 only) with the rotations
  // of earlier blocks applied; one thread per column.
  for (int j = tid; j < p; j += kSmallBlock) {
    const int c = i0 + j;
    double* h = Hr + (int64_t)c * ldh;
    for (int r = 0; r <= c + 1; ++r) h[r] = Hraw[(int64_t)c * ldh + r];
    for (int r = 0; r < i0; ++r) {
      const double a = h[r], b = h[r + 1];
      h[r] = cs[r] * a + sn[r] * b;
      h[r + 1] = -sn[r] * a + cs[r] * b;
    }
  }
  __syncthreads();
  // Rotations of this block, in order.
  __shared__ int stop;
  if (tid == 0) stop = 0;
  __syncthreads();
  int kdone = p, conv = 0, bad = 0;
  for (int j = 0; j < p; ++j) {
    const int c = i0 + j;
    double* h = Hr + (int64_t)c * ldh;
    if (tid == 0) {
      const double a = h[c], b = h[c + 1];
      double cc, ss, rr;
      if (b == 0.0) {
        cc = 1.0; ss = 0.0; rr = a;
      } else {
        rr = hypot(a, b);
        cc = a / rr;
        ss = b / rr;
      }
      cs[c] = cc;
      sn[c] = ss;
      h[c] = rr;
      h[c + 1] = 0.0;
      const double gc = g[c];
      g[c] = cc * gc;
      g[c + 1] = -ss * gc;
      const double res = fabs(g[c + 1]) / beta0[0];
      res_out[j] = res;
      if (!isfinite(res)) stop = 2;
      else if (res <= tol) stop = 1;
    }
    __syncthreads();
    if (stop) {
      kdone = j + 1;
      conv = stop == 1;
      bad = stop == 2;
      break;
    }
    // apply rotation c to the later columns of the block
    const double cc = cs[c], ss = sn[c];
    for (int jj = j + 1 + tid; jj < p; jj += kSmallBlock) {
      double* h2 = Hr + (int64_t)(i0 + jj) * ldh;
      const double a = h2[c], b = h2[c + 1];
      h2[c] = cc * a + ss * b;
      h2[c + 1] = -ss * a + cc * b;
    }
    __syncthreads();
  }
  if (tid == 0) {
    ctrl[C_KDONE] = kdone;
    ctrl[C_CONV] = conv;
    ctrl[C_BAD] = bad;
  }
}

// y = Hr(0:k, 0:k)^{-1} g(0:k), column-oriented back substitution.
__global__ __launch_bounds__(kSmallBlock) void k_back_solve(
    const double* __restrict__ Hr, int ldh, const double* __restrict__ g,
    int k, double* __restrict__ y) {
  __shared__ double b[4096];
  __shared__ double yj;
  for (int i = threadIdx.x; i < k; i += kSmallBlock) b[i] = g[i];
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    if (threadIdx.x == 0) {
      yj = b[j] / Hr[(int64_t)j * ldh + j];
      y[j] = yj;
    }
    __syncthreads();
    const double v = yj;
    for (int i = threadIdx.x; i < j; i += kSmallBlock)
      b[i] -= Hr[(int64_t)j * ldh + i] * v;
    __syncthreads();
  }
}

__global__ void k_givens_init(double* g, int m, const double* beta) {
  for (int i = threadIdx.x; i <= m; i += blockDim.x)
    g[i] = i == 0 ? beta[0] : 0.0;
}

}  // namespace

void pchol_ice(const double* G, int ldg, int smax, const int* s_dev,
               double omega, double* R, double* Rinv, int ldr, int* p_out,
               double* scratch, hipStream_t st) {
  hipLaunchKernelGGL(k_pchol, dim3(1), dim3(kSmallBlock), 0, st, G, ldg, smax,
                     s_dev, omega, R, Rinv, ldr, p_out, scratch);
  SGM_CHECK_LAUNCH();
}

void combine_r(const double* W, int ldw, const double* R2, int ldr2,
               const double* Z, const double* Zt, int ldz, int i, int* ctrl,
               double* Rtop, int ldt, double* Rkk, int ldk, hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3(1), dim3(kSmallBlock), 0, st, W, ldw, R2,
                     ldr2, Z, Zt, ldz, i, ctrl, Rtop, ldt, Rkk, ldk);
  SGM_CHECK_LAUNCH();
}

void hess_givens(double* Hraw, double* Hr, int ldh, double* cs, double* sn,
                 double* g, int nb, const double* Rtop, int ldt,
                 const double* Rkk, int ldk, const double* rec, int n_rec,
                 const double* beta0, double tol, int* ctrl, double* res_out,
                 double* /*scratch*/, hipStream_t st) {
  hipLaunchKernelGGL(k_hess_givens, dim3(1), dim3(kSmallBlock), 0, st, Hraw,
                     Hr, ldh, cs, sn, g, nb, Rtop, ldt, Rkk, ldk, rec, n_rec,
                     beta0, tol, ctrl, res_out);
  SGM_CHECK_LAUNCH();
}

void back_solve(const double* Hr, int ldh, const double* g, const int* /*kdev*/,
                int k, double* y, hipStream_t st) {
  if (k <= 0) return;
  if (k > 4096) throw Error{SGM_EINVAL, "restart length above 4096"};
  hipLaunchKernelGGL(k_back_solve, dim3(1), dim3(kSmallBlock), 0, st, Hr, ldh,
                     g, k, y);
  SGM_CHECK_LAUNCH();
}

void givens_init(double* g, int m, const double* beta, hipStream_t st) {
  hipLaunchKernelGGL(k_givens_init, dim3(1), dim3(256), 0, st, g, m, beta);
  SGM_CHECK_LAUNCH();
}

}  // namespace sgm
