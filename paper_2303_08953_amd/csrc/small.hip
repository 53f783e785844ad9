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

// Broadcast lane `lane`'s value of a double to the whole wavefront.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
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

// Partial Cholesky (Alg. 3) of the leading s x s block of G, right-looking,
// in LDS (row-major work copy).  Thread k owns column k (s <= blockDim.x).
// After the pivot of column j the incremental condition estimator takes its
// step.  The estimator keeps unit approximate singular vectors y (largest
// singular value, |y^T R|) and d = R^{-T} x (smallest, 1/|d|); column j's
// update is a 2x2 symmetric eigenproblem in (sin, cos) that needs
// a = y^T R(0:j, j) and a2 = d^T R(0:j, j).  Both are kept as running sums
// for every later column k: when row j of R appears, P_k <- s1 P_k +
// c1 R(j, k) and Q_k <- s2 Q_k + d_j R(j, k), which is exactly
// y^T R(0:j+1, k) and d^T R(0:j+1, k) after the update y <- [s1 y; c1],
// d <- [s2 d; d_j].  No reductions are needed.
// Pipeline of step j (several wavefronts):
//   (a) every thread reads the published estimator step of column j
//       (pivot root, its reciprocal, the two rotations, d_j, stop flag);
//   (b) the owners scale row j into rowj[], update their running sums, and
//       the owner of column j + 1 publishes (P, Q) and its next pivot
//       A(j+1, j+1) - R(j, j+1)^2;
//   (c) wavefront 0 evaluates the estimator step of column j + 1 while the
//       other wavefronts apply the rank-1 trailing update of row j.
// With one wavefront, (c) runs the estimator step and then the update.
// The factorisation stops before a column whose pivot is not positive and
// finite or whose estimate exceeds omega.  Outputs: p, R (p x p upper),
// Rinv = R^{-1}, both column-major with leading dimension ldr.
constexpr int kPcholLds = 140 * 1024 / 8;
constexpr int kPcholMaxS = 256;

// Estimator step of column j (all lanes of the calling wavefront): from the
// pivot and the running sums of column j, update (smax2, dn2) and return
// the step in e[0..7]: rjj, 1/rjj, s1, c1, s2, c2, d_j, stop (0/1); the
// same on every lane.
__device__ __forceinline__ void ice_eval(int j, double piv, double a,
                                         double a2, double omega,
                                         double& smax2, double& dn2,
                                         double* e) {
  const int lane = threadIdx.x % kWave;
  double stop = 0.0;
  double rjj = 0.0, rinv = 0.0, s1 = 0.0, c1 = 1.0, s2 = 0.0, c2 = 1.0;
  double dj = 0.0;
  if (!(piv > 0.0) || !isfinite(piv)) {
    stop = 1.0;
  } else {
    rjj = sqrt(piv);
    rinv = 1.0 / rjj;
    double kappa = 1.0;
    const double r2 = rjj * rjj;
    if (j == 0) {
      smax2 = r2;
      dn2 = rinv * rinv;
    } else {
      // the two 2x2 eigenproblems side by side: even lanes take the
      // largest singular value, odd lanes the smallest
      const bool second = lane & 1;
      const double ar = a2 * rinv;
      const double ea = second ? dn2 + ar * ar : smax2 + a * a;
      const double eb = second ? -ar * rinv : a * rjj;
      const double ec = second ? rinv * rinv : r2;
      double lam, u, v;
      top_eig_2x2(ea, eb, ec, lam, u, v);
      smax2 = readlane_f64(lam, 0);
      s1 = readlane_f64(u, 0);
      c1 = readlane_f64(v, 0);
      dn2 = readlane_f64(lam, 1);
      s2 = readlane_f64(u, 1);
      c2 = readlane_f64(v, 1);
      kappa = sqrt(smax2 * dn2);
    }
    if (!(kappa <= omega)) stop = 1.0;
    dj = (c2 - s2 * a2) * rinv;
  }
  e[0] = rjj;
  e[1] = rinv;
  e[2] = s1;
  e[3] = c1;
  e[4] = s2;
  e[5] = c2;
  e[6] = dj;
  e[7] = stop;
}

// The same, published in est[0..7] (LDS) for the other wavefronts.
__device__ __forceinline__ void ice_step(int j, double piv, double a,
                                         double a2, double omega,
                                         double& smax2, double& dn2,
                                         double* est) {
  double e[8];
  ice_eval(j, piv, a, a2, omega, smax2, dn2, e);
  if (threadIdx.x % kWave == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) est[k] = e[k];
}

// The body is instantiated twice: with the LDS array (every access then
// compiles to a ds_* instruction) and with global scratch for large s.
__device__ __forceinline__ void pchol_body(
    double* Aw, double* rowj, double (*bc)[3], double (*est)[8],
    const double* __restrict__ G, int ldg, int s, double omega,
    double* __restrict__ R, double* __restrict__ Rinv, int ldr, int* p_out) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int lane = tid % kWave, wave = tid / kWave, nw = nthr / kWave;
  const int la = s > 0 ? s : 1;
  // Rinv rows padded to an odd stride: the column sweep below has each
  // thread walk its own row, and an even stride would put all of them in
  // one LDS bank
  const int lri = s + 1;
  double* Ri = Aw + (size_t)s * s;
  // G symmetric: (i, j) -> row i, col j; eight loads in flight per thread
  for (int e0 = tid; e0 < s * s; e0 += 8 * nthr) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nthr;
      const int i = e % la, j = e / la;
      v[q] = e < s * s ? G[(int64_t)j * ldg + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nthr;
      const int i = e % la, j = e / la;
      if (e < s * s) Aw[i * la + j] = v[q];
    }
  }
  double P = 0.0, Q = 0.0;        // estimator sums of column tid
  double smax2 = 0.0, dn2 = 0.0;  // estimator state (wavefront 0)
  int p = s;
  __syncthreads();
  if (s > 0 && wave == 0)
    ice_step(0, Aw[0], 0.0, 0.0, omega, smax2, dn2, est[0]);
  __syncthreads();
  // trailing update of row j over the given wavefronts
  auto trail = [&](int j, int w0, int nwu) {
    for (int k = j + 1 + lane; k < s; k += kWave) {
      const double rk = rowj[k];
      int l = j + 1 + (wave - w0);
      for (; l + 3 * nwu <= k; l += 4 * nwu) {
        double* a = Aw + (size_t)l * la + k;
        const size_t st = (size_t)nwu * la;
        const double a0 = a[0], a1 = a[st], a2 = a[2 * st], a3 = a[3 * st];
        const double r0 = rowj[l], r1 = rowj[l + nwu], r2 = rowj[l + 2 * nwu],
                     r3 = rowj[l + 3 * nwu];
        a[0] = a0 - r0 * rk;
        a[st] = a1 - r1 * rk;
        a[2 * st] = a2 - r2 * rk;
        a[3 * st] = a3 - r3 * rk;
      }
      for (; l <= k; l += nwu) Aw[(size_t)l * la + k] -= rowj[l] * rk;
    }
  };
  for (int j = 0; j < s; ++j) {
    // (a) the estimator step of column j
    const double* e = est[j & 1];
    if (e[7] != 0.0) { p = j; break; }
    const double rjj = e[0], rinv = e[1], s1 = e[2], c1 = e[3], s2 = e[4],
                 dj = e[6];
    // (b) row j of R, the running sums, and what the next step needs
    if (tid > j && tid < s) {
      const double rjk = Aw[j * la + tid] * rinv;
      Aw[j * la + tid] = rjk;
      rowj[tid] = rjk;
      P = s1 * P + c1 * rjk;
      Q = s2 * Q + dj * rjk;
      if (tid == j + 1) {
        bc[(j + 1) & 1][0] = P;
        bc[(j + 1) & 1][1] = Q;
        bc[(j + 1) & 1][2] = Aw[(j + 1) * la + j + 1] - rjk * rjk;
      }
    }
    if (tid == j) Aw[j * la + j] = rjj;
    __syncthreads();
    // (c) next estimator step beside the trailing update
    const bool more = j + 1 < s;
    if (nw == 1) {
      if (more) {
        const double* b = bc[(j + 1) & 1];
        ice_step(j + 1, b[2], b[0], b[1], omega, smax2, dn2,
                 est[(j + 1) & 1]);
      }
      trail(j, 0, 1);
    } else if (wave == 0) {
      if (more) {
        const double* b = bc[(j + 1) & 1];
        ice_step(j + 1, b[2], b[0], b[1], omega, smax2, dn2,
                 est[(j + 1) & 1]);
      }
    } else {
      trail(j, 1, nw - 1);
    }
    __syncthreads();
  }
  if (tid == 0) *p_out = p;
  // Rinv by recursive doubling: the diagonal holds 1 / R(i, i); at level b
  // neighbouring inverted diagonal blocks A^{-1} (rows a0..a0+b) and
  // C^{-1} (rows c0 = a0+b ..) of the factor [A B; 0 C] are joined through
  // the off-diagonal block -A^{-1} (B C^{-1}): two products, every output
  // in parallel, log2(p) levels.  T = B C^{-1} is kept, transposed, in the
  // unused lower triangle of the same block pair.
  for (int i = tid; i < p; i += nthr) Ri[i * lri + i] = 1.0 / Aw[i * la + i];
  __syncthreads();
  for (int b = 1; b < p; b *= 2) {
    const int npairs = (p + 2 * b - 1) / (2 * b);
    const int items = npairs * b * b;
    for (int e = tid; e < items; e += nthr) {   // T = B C^{-1}
      const int q = e / (b * b), i = (e % (b * b)) / b, j = e % b;
      const int a0 = 2 * q * b, c0 = a0 + b;
      if (c0 + j >= p) continue;
      double acc = 0.0;
      for (int t = 0; t <= j; ++t)
        acc += Aw[(a0 + i) * la + c0 + t] * Ri[(c0 + t) * lri + c0 + j];
      Ri[(c0 + j) * lri + a0 + i] = acc;  // transposed, lower triangle
    }
    __syncthreads();
    for (int e = tid; e < items; e += nthr) {   // X = -A^{-1} T
      const int q = e / (b * b), i = (e % (b * b)) / b, j = e % b;
      const int a0 = 2 * q * b, c0 = a0 + b;
      if (c0 + j >= p) continue;
      double acc = 0.0;
      for (int t = i; t < b; ++t)
        acc += Ri[(a0 + i) * lri + a0 + t] * Ri[(c0 + j) * lri + a0 + t];
      Ri[(a0 + i) * lri + c0 + j] = -acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < p * p; e += nthr) {
    const int i = e % p, j = e / p;
    const bool up = i <= j;
    R[(int64_t)j * ldr + i] = up ? Aw[i * la + j] : 0.0;
    Rinv[(int64_t)j * ldr + i] = up ? Ri[i * lri + j] : 0.0;
  }
}

__global__ __launch_bounds__(kSmallBlock) void k_pchol(
    const double* __restrict__ G, int ldg, int smax, const int* s_dev,
    double omega, double* __restrict__ R, double* __restrict__ Rinv, int ldr,
    int* p_out, double* scratch) {
  __shared__ double buf[kPcholLds];
  __shared__ double rowj[kPcholMaxS];
  __shared__ double bc[2][3];
  __shared__ double est[2][8];
  int s = smax;
  if (s_dev) s = min(s, *s_dev);
  // work layout: A (s x s, row-major) | Rinv (s x (s + 1), row-major)
  if ((size_t)s * (2 * s + 1) <= (size_t)kPcholLds)
    pchol_body(buf, rowj, bc, est, G, ldg, s, omega, R, Rinv, ldr, p_out);
  else
    pchol_body(scratch, rowj, bc, est, G, ldg, s, omega, R, Rinv, ldr, p_out);
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

// C(0:m, 0:n) = (add ? C : 0) + alpha A(0:m, 0:k) B(0:k, 0:n), column-major
// operands in LDS or global memory, on the float64 matrix cores
// (v_mfma_f64_16x16x4f64): the block's wavefronts take 16 x 16 output
// tiles in turn; lane l supplies A(m0 + l % 16, k0 + l / 16) and
// B(k0 + l / 16, n0 + l % 16) per 4-deep step (zero outside the operands)
// and holds C(m0 + l / 16 + 4 j, n0 + l % 16) in result register j.  Each
// output is a fixed-order sum over k.
__device__ __forceinline__ void tile_gemm_mfma(int m, int n, int k,
                                               const double* A, int lda,
                                               const double* B, int ldb,
                                               double* C, int ldc,
                                               double alpha, bool add) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int TM = (m + 15) / 16, TN = (n + 15) / 16;
  for (int t = wave; t < TM * TN; t += nw) {
    const int m0 = (t % TM) * 16, n0 = (t / TM) * 16;
    const int ra = m0 + c16, cb = n0 + c16;
    const bool ina = ra < m, inb = cb < n;
    const double* ap = A + (ina ? ra : 0);
    const double* bp = B + (size_t)(inb ? cb : 0) * ldb;
    auto lda_at = [&](int kk) {
      return (ina && kk < k) ? ap[(size_t)kk * lda] : 0.0;
    };
    auto ldb_at = [&](int kk) { return (inb && kk < k) ? bp[kk] : 0.0; };
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    // eight steps' operands are loaded together (an operand in global
    // memory would otherwise cost its full latency per step)
    for (int k0 = 0; k0 < k; k0 += 32) {
      double a[8], b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = lda_at(k0 + 4 * q + g);
        b[q] = ldb_at(k0 + 4 * q + g);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + 4 * q < k)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = m0 + g + 4 * j;
      if (r < m && inb) {
        double* cp = C + (size_t)cb * ldc + r;
        *cp = (add ? *cp : 0.0) + alpha * acc[j];
      }
    }
  }
}

// Fused tail of one block (one workgroup).
//  1. Combine the BCGS passes (Alg. 4): R(1:nb, k) = W + R2 Z and
//     R(k, k) = Zt Z (Z, Zt upper triangular).
//  2. Hessenberg recovery: with Rt = [e_nb | R(1:nb+p, k)] and the
//     (p+1) x p change-of-basis matrix B of the recurrence records,
//     H(1:nb+p, nb:nb+p-1) = (Rt B - [H(1:nb, 1:nb-1) X; 0]) T^{-1},
//     X = Rt(1:nb-1, :), T = Rt(nb:nb+p-1, :) = [1 a^T; 0 R(k,k)'] where
//     R(k,k)' is the leading (p-1) block, so T^{-1} = [1 -a^T K; 0 K] with
//     K = R(k,k)'^{-1} = (Z^{-1} Zt^{-1})' from the two explicit inverses.
//  3. Givens: the earlier rotations on the new columns, then the new ones in
//     order with the relative residual estimate |g(c+1)| / beta0 and the
//     convergence test after every column.
// Work in LDS (global scratch when it does not fit); the small products are
// register-tiled; the rotation sweeps run on wavefront 0 with each lane
// owning whole columns.  A breakdown (p2 = 0) yields one column with a zero
// subdiagonal.
constexpr int kTailLds = 150 * 1024 / 8;
constexpr int kTailMaxP = 256;  // largest block

// doubles of the work area:
//   Rt_top nb*p | Rkk p*p | Tinv p*p | union(R2 nb*p, Z, Zt, Zi, Zti p*p
//   each ; Mb nr*p) | Hn nr*p | css nb | sns nb | gs p+1 | pad
// The union's inputs are dead once step 1 has finished.
__host__ __device__ inline size_t tail_union(int nb, int p) {
  const size_t a = (size_t)nb * p + 4 * (size_t)p * p;
  const size_t b = (size_t)(nb + p) * p;
  return a > b ? a : b;
}
__host__ __device__ inline size_t tail_doubles(int nb, int p) {
  return (size_t)nb * p + 2 * (size_t)p * p + tail_union(nb, p) +
         (size_t)(nb + p) * p + 2 * (size_t)nb + (size_t)p + 16;
}

__device__ __forceinline__ void tail_body(
    double* base, int* sh, const double* __restrict__ W,
    const double* __restrict__ R2g, int ldw, const double* __restrict__ Zg,
    const double* __restrict__ Ztg, const double* __restrict__ Zig,
    const double* __restrict__ Ztig, int ldz, int nb, int* ctrl,
    double* __restrict__ Rtop_out, double* __restrict__ Rkk_out,
    double* __restrict__ Hraw, double* __restrict__ Hr, int ldh,
    double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
    const double* __restrict__ rec, int n_rec,
    const double* __restrict__ beta0, double tol,
    double* __restrict__ res_out, int* __restrict__ host_ctrl, int* stop,
    int seq, double* recs) {
  int& kdone_s = sh[0];
  int& conv_s = sh[1];
  int& bad_s = sh[2];
  const int tid = threadIdx.x;
  const int p1 = ctrl[C_P1], p2 = ctrl[C_P2];
  const bool brk = p2 == 0;
  const int p = brk ? 1 : p2;
  const int pz = brk ? (p1 > 0 ? 1 : 0) : p;  // columns of R2 / Z used
  const int i0 = nb - 1;
  const int nr = nb + p;  // rows of the new block
  double* Rt_top = base;                   // nb x p
  double* Rkk = Rt_top + (size_t)nb * p;   // p x p
  double* Tinv = Rkk + (size_t)p * p;      // p x p
  double* uni = Tinv + (size_t)p * p;
  double* R2 = uni;                        // nb x p
  double* Z = R2 + (size_t)nb * p;         // p x p each
  double* Zt = Z + (size_t)p * p;
  double* Zi = Zt + (size_t)p * p;
  double* Zti = Zi + (size_t)p * p;
  double* Mb = uni;                        // nr x p (after step 1)
  double* Hn = uni + tail_union(nb, p);    // nr x p
  double* css = Hn + (size_t)nr * p;
  double* sns = css + nb;
  double* gs = sns + nb;
  // 0. stage the inputs (coalesced, with a batch of loads in flight per
  // thread: one global round trip per batch instead of one per element);
  // Z, Zt, Zi, Zti zero-padded to p x p; the recurrence records of the p
  // new columns
  {
    const int nbp = nb * p;
    for (int e0 = tid; e0 < nbp; e0 += 8 * kSmallBlock) {
      double v[8], u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + q * kSmallBlock;
        const int r = e % nb, c = e / nb;
        const bool in = e < nbp;
        v[q] = in && c < pz && p1 > 0 ? R2g[(int64_t)c * ldw + r] : 0.0;
        u[q] = in ? W[(int64_t)c * ldw + r] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + q * kSmallBlock;
        const int r = e % nb, c = e / nb;
        if (e < nbp) {
          R2[(size_t)c * nb + r] = v[q];
          Rt_top[(size_t)c * nb + r] = u[q];
        }
      }
    }
    const int pp = p * p;
    for (int e0 = tid; e0 < pp; e0 += 4 * kSmallBlock) {
      double z[4], zt[4], zi[4], zti[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * kSmallBlock;
        const int r = e % p, c = e / p;
        const bool in = e < pp && r < pz && c < pz;
        const bool in2 = e < pp && !brk;
        const int64_t o = (int64_t)c * ldz + r;
        z[q] = in ? Zg[o] : 0.0;
        zt[q] = in2 ? Ztg[o] : 0.0;
        zi[q] = in2 ? Zig[o] : 0.0;
        zti[q] = in2 ? Ztig[o] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * kSmallBlock;
        if (e < pp) {
          Z[e] = z[q];
          Zt[e] = zt[q];
          Zi[e] = zi[q];
          Zti[e] = zti[q];
        }
      }
    }
    for (int r0 = tid; r0 < i0; r0 += 4 * kSmallBlock) {
      double c4[4], s4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + q * kSmallBlock;
        c4[q] = r < i0 ? cs[r] : 0.0;
        s4[q] = r < i0 ? sn[r] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + q * kSmallBlock;
        if (r < i0) {
          css[r] = c4[q];
          sns[r] = s4[q];
        }
      }
    }
    for (int j = tid; j < p; j += kSmallBlock) {
      const int q = j % n_rec;
      recs[3 * j] = rec[3 * q];
      recs[3 * j + 1] = rec[3 * q + 1];
      recs[3 * j + 2] = rec[3 * q + 2];
    }
  }
  if (tid == 0) {
    ctrl[C_PH] = p;
    ctrl[C_BREAK] = brk ? 1 : 0;
  }
  __syncthreads();
  // 1. combine: Rt_top = W + R2 Z, Rkk = Zt Z
  tile_gemm_mfma(nb, p, p, R2, nb, Z, p, Rt_top, nb, 1.0, true);
  tile_gemm_mfma(p, p, p, Zt, p, Z, p, Rkk, p, 1.0, false);
  // K = (Zi Zti)' into Tinv(1:p, 1:p)
  if (p > 1) tile_gemm_mfma(p - 1, p - 1, p - 1, Zi, p, Zti, p, Tinv + p + 1, p,
                       1.0, false);
  __syncthreads();
  if (Rtop_out)
    for (int e = tid; e < nb * p; e += kSmallBlock) {
      const int r = e % nb, c = e / nb;
      Rtop_out[(int64_t)c * ldw + r] = Rt_top[(size_t)c * nb + r];
    }
  if (Rkk_out)
    for (int e = tid; e < p * p; e += kSmallBlock) {
      const int r = e % p, c = e / p;
      Rkk_out[(int64_t)c * ldz + r] = Rkk[(size_t)c * p + r];
    }
  // first row and column of T^{-1}: [1, -a^T K], a = Rt(i0, 1:p-1)
  for (int c = tid; c < p; c += kSmallBlock) {
    double v;
    if (c == 0) {
      v = 1.0;
    } else {
      double acc = 0.0;
#pragma unroll 8
      for (int t = 0; t < p - 1; ++t)
        acc += Rt_top[(size_t)t * nb + i0] * Tinv[(size_t)c * p + 1 + t];
      v = -acc;
    }
    Tinv[(size_t)c * p] = v;
    if (c > 0) Tinv[c] = 0.0;
  }
  auto Rt = [&](int r, int c) -> double {  // nr x (p + 1)
    if (c == 0) return r == i0 ? 1.0 : 0.0;
    if (r < nb) return Rt_top[(size_t)(c - 1) * nb + r];
    return Rkk[(size_t)(c - 1) * p + (r - nb)];
  };
  // 2. M = Rt B (tridiagonal B from the records), then M(1:nb, 2:p) -= H X
  for (int e = tid; e < nr * p; e += kSmallBlock) {
    const int r = e % nr, j = e / nr;
    const double th = recs[3 * j], ga = recs[3 * j + 1], de = recs[3 * j + 2];
    double m = th * Rt(r, j) + ga * Rt(r, j + 1);
    if (j >= 1) m += de * Rt(r, j - 1);
    Mb[(size_t)j * nr + r] = m;
  }
  __syncthreads();
  if (nb > 1 && p > 1)
    tile_gemm_mfma(nb, p - 1, i0, Hraw, ldh, Rt_top, nb, Mb + nr, nr, -1.0, true);
  __syncthreads();
  // Hn = M T^{-1}; write the new columns of H
  tile_gemm_mfma(nr, p, p, Mb, nr, Tinv, p, Hn, nr, 1.0, false);
  __syncthreads();
  for (int e = tid; e < nr * p; e += kSmallBlock) {
    const int r = e % nr, j = e / nr;
    Hraw[(int64_t)(i0 + j) * ldh + r] = Hn[(size_t)j * nr + r];
  }
  // 3. rotations on wavefront 0: lane l owns columns l, l + 64, ...
  if (tid < kWave) {
    const int lane = tid;
    // earlier rotations on every new column (rows <= c + 1 only); the
    // rotated pair's lower entry is carried in a register
    for (int j = lane; j < p; j += kWave) {
      double* h = Hn + (size_t)j * nr;
      if (i0 > 0) {
        double carry = h[0];
        int r = 0;
        // eight rows per batch: the loads go out before the dependent chain
        for (; r + 8 <= i0; r += 8) {
          double b[8], c0[8], s0[8], o[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            b[q] = h[r + 1 + q];
            c0[q] = css[r + q];
            s0[q] = sns[r + q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            o[q] = c0[q] * carry + s0[q] * b[q];
            carry = -s0[q] * carry + c0[q] * b[q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) h[r + q] = o[q];
        }
        for (; r < i0; ++r) {
          const double b = h[r + 1], c0 = css[r], s0 = sns[r];
          h[r] = c0 * carry + s0 * b;
          carry = -s0 * carry + c0 * b;
        }
        h[i0] = carry;
      }
    }
    // new rotations in order; g's running entry gcur is uniform.  Lane l
    // keeps, for each of its columns jj = l + 64 q, the entry at the
    // current rotation row c in cur[q] and the next row's entry in nxt[q]
    // and the one after in nx2[q] (read two rows ahead from LDS, so the
    // owner's operands are in registers when its turn comes): rotation
    // j needs only the owner's two registers, and applying it to a later
    // column leaves that column's row c final (stored) and its row c + 1
    // in cur.  The rotation chain per column then holds no LDS round trip.
    constexpr int NQ = kTailMaxP / kWave;
    double cur[NQ], nxt[NQ], nx2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int jj = lane + kWave * q;
      const bool in = jj < p;
      cur[q] = in ? Hn[(size_t)jj * nr + i0] : 0.0;
      nxt[q] = in ? Hn[(size_t)jj * nr + i0 + 1] : 0.0;
      nx2[q] = in && i0 + 2 < nr ? Hn[(size_t)jj * nr + i0 + 2] : 0.0;
    }
    double gcur = g[i0];
    const double b0 = beta0[0];
    int kdone = p, conv = 0, bad = 0;
    for (int j = 0; j < p; ++j) {
      const int c = i0 + j;
      const int owner = j % kWave, qo = j / kWave;
      double cc = 1.0, ss = 0.0;
      if (lane == owner) {
        double a = cur[0], b = nxt[0];
#pragma unroll
        for (int q = 1; q < NQ; ++q)
          if (q == qo) {
            a = cur[q];
            b = nxt[q];
          }
        double rr = a;
        if (b != 0.0) {
          rr = hypot(a, b);
          cc = a / rr;
          ss = b / rr;
        }
        double* h = Hn + (size_t)j * nr;
        h[c] = rr;
        h[c + 1] = 0.0;
      }
      cc = readlane_f64(cc, owner);
      ss = readlane_f64(ss, owner);
      const double gnew = -ss * gcur;
      const double res = fabs(gnew) / b0;
      if (lane == 0) {
        cs[c] = cc;
        sn[c] = ss;
        gs[j] = cc * gcur;
        res_out[j] = res;
      }
      gcur = gnew;
      if (!isfinite(res) || res <= tol) {
        kdone = j + 1;
        conv = isfinite(res) ? 1 : 0;
        bad = isfinite(res) ? 0 : 1;
        break;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int jj = lane + kWave * q;
        if (jj > j && jj < p) {
          double* h2 = Hn + (size_t)jj * nr;
          const double a = cur[q], b = nxt[q];
          h2[c] = cc * a + ss * b;
          cur[q] = -ss * a + cc * b;
          nxt[q] = nx2[q];
          nx2[q] = c + 3 < nr ? h2[c + 3] : 0.0;
        }
      }
    }
    if (lane == 0) {
      gs[kdone] = gcur;
      kdone_s = kdone;
      conv_s = conv;
      bad_s = bad;
    }
  }
  __syncthreads();
  const int kdone = kdone_s;
  // write back the rotated columns (rows <= c + 1) and g
  for (int e = tid; e < kdone * nr; e += kSmallBlock) {
    const int j = e / nr, r = e % nr;
    const int c = i0 + j;
    if (r <= c + 1) Hr[(int64_t)c * ldh + r] = Hn[(size_t)j * nr + r];
  }
  for (int r = tid; r <= kdone; r += kSmallBlock) g[i0 + r] = gs[r];
  if (tid == 0) {
    ctrl[C_KDONE] = kdone;
    ctrl[C_CONV] = conv_s;
    ctrl[C_BAD] = bad_s;
    // the gate of matrix powers steps queued for the next block
    ctrl[C_GO] = (brk || conv_s || bad_s) ? -1 : p2;
    // the control words the host needs, straight into its mapped memory
    if (host_ctrl)
      for (int k = 0; k < C_NCTRL; ++k) host_ctrl[k] = ctrl[k];
    if (stop && (brk || conv_s || bad_s)) *stop = 1;
    // then the sequence word, once the estimates and control words (all
    // written by this thread) are visible to the host
    if (host_ctrl && seq > 0) {
      __threadfence_system();
      __hip_atomic_store(host_ctrl + kSeqWord, seq, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__global__ __launch_bounds__(kSmallBlock) void k_block_tail(
    const double* __restrict__ W, const double* __restrict__ R2g, int ldw,
    const double* __restrict__ Zg, const double* __restrict__ Ztg,
    const double* __restrict__ Zig, const double* __restrict__ Ztig, int ldz,
    int nb, int* ctrl, double* __restrict__ Rtop_out,
    double* __restrict__ Rkk_out, double* __restrict__ Hraw,
    double* __restrict__ Hr, int ldh, double* __restrict__ cs,
    double* __restrict__ sn, double* __restrict__ g,
    const double* __restrict__ rec, int n_rec,
    const double* __restrict__ beta0, double tol, double* __restrict__ res_out,
    int* __restrict__ host_ctrl, double* scratch, int* stop, int seq) {
  __shared__ double lds[kTailLds];
  __shared__ double recs[3 * kTailMaxP];  // records of the new columns
  __shared__ int sh[4];
  // a queued step after the end of the cycle: leave every state untouched
  // (the flag was written by an earlier kernel of the stream)
  if (stop && *stop) return;
  const int p = ctrl[C_P2] == 0 ? 1 : ctrl[C_P2];
  if (tail_doubles(nb, p) <= (size_t)kTailLds)
    tail_body(lds, sh, W, R2g, ldw, Zg, Ztg, Zig, Ztig, ldz, nb, ctrl,
              Rtop_out, Rkk_out, Hraw, Hr, ldh, cs, sn, g, rec, n_rec, beta0,
              tol, res_out, host_ctrl, stop, seq, recs);
  else
    tail_body(scratch, sh, W, R2g, ldw, Zg, Ztg, Zig, Ztig, ldz, nb, ctrl,
              Rtop_out, Rkk_out, Hraw, Hr, ldh, cs, sn, g, rec, n_rec, beta0,
              tol, res_out, host_ctrl, stop, seq, recs);
}

// y = Hr(0:k, 0:k)^{-1} g(0:k), column-oriented back substitution.
// Every thread first stages the upper triangle into LDS (packed by columns:
// column j's rows 0..j at j (j + 1) / 2), so the global latency is paid
// once; wavefront 0 then runs the k sequential steps with the right-hand
// side in registers (lane l holds rows l, l + 64, ...), broadcasting y_j
// from its owner lane.  NQ = rows per lane; the triangle is read from
// global memory when it does not fit in LDS.
constexpr int kBackLds = 150 * 1024 / 8;
constexpr int kBackThreads = 1024;

template <int NQ>
__device__ __forceinline__ void back_solve_wave(const double* T, bool packed,
                                                const double* __restrict__ Hr,
                                                int ldh,
                                                const double* __restrict__ g,
                                                int k, double* __restrict__ y) {
  const int lane = threadIdx.x;
  double b[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = lane + kWave * q;
    b[q] = i < k ? g[i] : 0.0;
  }
  auto t = [&](int i, int j) -> double {
    return packed ? T[(int64_t)j * (j + 1) / 2 + i] : Hr[(int64_t)j * ldh + i];
  };
  for (int j = k - 1; j >= 0; --j) {
    const int owner = j % kWave, qj = j / kWave;
    double bj = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q == qj) bj = b[q];
    const double yj = readlane_f64(bj, owner) / t(j, j);
    if (lane == 0) y[j] = yj;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + kWave * q;
      if (q <= qj && i < j) b[q] -= t(i, j) * yj;
    }
  }
}

__global__ __launch_bounds__(kBackThreads) void k_back_solve(
    const double* __restrict__ Hr, int ldh, const double* __restrict__ g,
    int k, double* __restrict__ y) {
  __shared__ double T[kBackLds];
  const int64_t npk = (int64_t)k * (k + 1) / 2;
  const bool packed = npk <= kBackLds;
  if (packed) {
    // column-major walk of the full k x k block; rows above the diagonal
    // are kept
#pragma unroll 4
    for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += kBackThreads) {
      const int j = (int)(e / k), i = (int)(e % k);
      if (i <= j) T[(int64_t)j * (j + 1) / 2 + i] = Hr[(int64_t)j * ldh + i];
    }
  }
  __syncthreads();
  if (threadIdx.x >= kWave) return;
  if (k <= 2 * kWave)
    back_solve_wave<2>(T, packed, Hr, ldh, g, k, y);
  else if (k <= 4 * kWave)
    back_solve_wave<4>(T, packed, Hr, ldh, g, k, y);
  else if (k <= 8 * kWave)
    back_solve_wave<8>(T, packed, Hr, ldh, g, k, y);
  else {
    // long cycles: the right-hand side lives in LDS (the triangle does not
    // fit there anyway)
    double* b = T;
    for (int i = threadIdx.x; i < k; i += kWave) b[i] = g[i];
    for (int j = k - 1; j >= 0; --j) {
      const double yj = b[j] / Hr[(int64_t)j * ldh + j];
      if (threadIdx.x == 0) y[j] = yj;
      for (int i = threadIdx.x; i < j; i += kWave)
        b[i] -= Hr[(int64_t)j * ldh + i] * yj;
    }
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
  // thread k owns column k; four wavefronts share the trailing updates
  const int threads = smax <= 8 ? kWave : kSmallBlock;
  if (smax > kPcholMaxS || smax > threads)
    throw Error{SGM_EINVAL, "partial Cholesky: block larger than 256"};
  hipLaunchKernelGGL(k_pchol, dim3(1), dim3(threads), 0, st, G, ldg, smax,
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

size_t block_tail_scratch_doubles(int nb_max, int s_max) {
  return tail_doubles(nb_max, s_max);
}

void block_tail(const double* W, const double* R2, int ldw, const double* Z,
                const double* Zt, const double* Zi, const double* Zti, int ldz,
                int nb, int* ctrl, double* Rtop, double* Rkk, double* Hraw,
                double* Hr, int ldh, double* cs, double* sn, double* g,
                const double* rec, int n_rec, const double* beta0, double tol,
                double* res_out, int* host_ctrl, double* scratch,
                hipStream_t st, int* stop, int seq) {
  hipLaunchKernelGGL(k_block_tail, dim3(1), dim3(kSmallBlock), 0, st, W, R2,
                     ldw, Z, Zt, Zi, Zti, ldz, nb, ctrl, Rtop, Rkk, Hraw, Hr,
                     ldh, cs, sn, g, rec, n_rec, beta0, tol, res_out,
                     host_ctrl, scratch, stop, seq);
  SGM_CHECK_LAUNCH();
}

void back_solve(const double* Hr, int ldh, const double* g, const int* /*kdev*/,
                int k, double* y, hipStream_t st) {
  if (k <= 0) return;
  if (k > 4096) throw Error{SGM_EINVAL, "restart length above 4096"};
  hipLaunchKernelGGL(k_back_solve, dim3(1), dim3(kBackThreads), 0, st, Hr,
                     ldh, g, k, y);
  SGM_CHECK_LAUNCH();
}

void givens_init(double* g, int m, const double* beta, hipStream_t st) {
  hipLaunchKernelGGL(k_givens_init, dim3(1), dim3(256), 0, st, g, m, beta);
  SGM_CHECK_LAUNCH();
}

}  // namespace sgm
