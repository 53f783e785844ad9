// Basis shifts on the GPU (Sec. 3.4 - 3.5): Ritz values of the pre-phase
// Hessenberg matrix by the Francis double-shift QR iteration, modified Leja
// ordering, the (scaled) Newton recurrence records and the initial
// step-size estimator of Eq. (auxiliarymatrix).  All float64, each kernel
// one workgroup.
#include "internal.h"

namespace sgm {

namespace {

// ------------------------------------------------------------------ HQR
// Eigenvalues of an upper Hessenberg matrix by implicitly double-shifted QR
// (Francis steps with 3x3 Householder reflectors, Golub & Van Loan,
// Sec. 7.5), working on the unreduced active window only since only
// eigenvalues are needed.  One wavefront: scalars are computed redundantly
// by every lane; reflector applications are split over the lanes.
constexpr int kHqrMax = 128;  // window held in LDS up to this order

__device__ __forceinline__ double& at(double* H, int ld, int r, int c) {
  return H[(int64_t)c * ld + r];
}

__device__ void house3(double x, double y, double z, double& v0, double& v1,
                       double& v2, double& beta) {
  const double nrm = sqrt(x * x + y * y + z * z);
  if (nrm == 0.0) {
    v0 = 1.0; v1 = 0.0; v2 = 0.0; beta = 0.0;
    return;
  }
  const double alpha = x >= 0.0 ? -nrm : nrm;
  v0 = x - alpha;
  v1 = y;
  v2 = z;
  const double vv = v0 * v0 + v1 * v1 + v2 * v2;
  beta = vv > 0.0 ? 2.0 / vv : 0.0;
}

__device__ void eig2(double a, double b, double c, double d, double& r1,
                     double& i1, double& r2, double& i2) {
  // eigenvalues of [[a, b], [c, d]] = d + p +- sqrt(p^2 + b c), p = (a-d)/2
  const double p = 0.5 * (a - d);
  const double disc = p * p + b * c;
  if (disc >= 0.0) {
    const double r = sqrt(disc);
    const double z = p >= 0.0 ? p + r : p - r;
    r1 = d + z;
    r2 = z != 0.0 ? d - (b * c) / z : d;
    i1 = 0.0;
    i2 = 0.0;
  } else {
    r1 = r2 = d + p;
    i1 = sqrt(-disc);
    i2 = -i1;
  }
}

__device__ __forceinline__ void hqr_body(double* H, int ld,
                                         const double* __restrict__ Hin,
                                         int ldh, int n, double* wr,
                                         double* wi, int* status) {
  const int lane = threadIdx.x;
  for (int e = lane; e < n * n; e += kWave) {
    const int r = e % n, c = e / n;
    at(H, ld, r, c) = r <= c + 1 ? Hin[(int64_t)c * ldh + r] : 0.0;
  }
  __syncthreads();
  double anorm = 0.0;
  for (int c = 0; c < n; ++c)
    for (int r = 0; r <= min(c + 1, n - 1); ++r) anorm += fabs(at(H, ld, r, c));
  const double ulp = 2.220446049250313e-16;
  int hi = n - 1;
  int its = 0, total = 0;
  int ok = 1;
  while (hi >= 0) {
    // deflation: find the start lo of the unreduced window ending at hi
    int lo = hi;
    while (lo > 0) {
      double s = fabs(at(H, ld, lo - 1, lo - 1)) + fabs(at(H, ld, lo, lo));
      if (s == 0.0) s = anorm;
      if (fabs(at(H, ld, lo, lo - 1)) <= ulp * s) break;
      --lo;
    }
    __syncthreads();
    if (lo > 0 && lane == 0) at(H, ld, lo, lo - 1) = 0.0;
    if (lo == hi) {
      if (lane == 0) { wr[hi] = at(H, ld, hi, hi); wi[hi] = 0.0; }
      hi -= 1;
      its = 0;
      __syncthreads();
      continue;
    }
    if (lo == hi - 1) {
      double r1, i1, r2, i2;
      eig2(at(H, ld, hi - 1, hi - 1), at(H, ld, hi - 1, hi),
           at(H, ld, hi, hi - 1), at(H, ld, hi, hi), r1, i1, r2, i2);
      if (lane == 0) {
        wr[hi - 1] = r1; wi[hi - 1] = i1;
        wr[hi] = r2; wi[hi] = i2;
      }
      hi -= 2;
      its = 0;
      __syncthreads();
      continue;
    }
    if (++total > 40 * n) { ok = 0; break; }
    ++its;
    // shifts: eigenvalues of the trailing 2x2 (sum s, product t), or an
    // exceptional pair after 10 and 20 stagnant steps
    double s, t;
    const double hmm = at(H, ld, hi - 1, hi - 1), hnn = at(H, ld, hi, hi);
    if (its == 10 || its == 20) {
      const double w = fabs(at(H, ld, hi, hi - 1)) + fabs(at(H, ld, hi - 1, hi - 2));
      const double sh = hnn + 0.75 * w;
      s = 2.0 * sh;
      t = sh * sh + 0.25 * w * w;
    } else {
      s = hmm + hnn;
      t = hmm * hnn - at(H, ld, hi - 1, hi) * at(H, ld, hi, hi - 1);
    }
    double x = at(H, ld, lo, lo) * at(H, ld, lo, lo) +
               at(H, ld, lo, lo + 1) * at(H, ld, lo + 1, lo) -
               s * at(H, ld, lo, lo) + t;
    double y = at(H, ld, lo + 1, lo) *
               (at(H, ld, lo, lo) + at(H, ld, lo + 1, lo + 1) - s);
    double z = at(H, ld, lo + 1, lo) * at(H, ld, lo + 2, lo + 1);
    for (int k = lo; k <= hi - 2; ++k) {
      double v0, v1, v2, beta;
      house3(x, y, z, v0, v1, v2, beta);
      const int c0 = k > lo ? k - 1 : lo;
      __syncthreads();
      // left: rows k..k+2, columns c0..hi
      for (int c = c0 + lane; c <= hi; c += kWave) {
        const double a0 = at(H, ld, k, c), a1 = at(H, ld, k + 1, c),
                     a2 = at(H, ld, k + 2, c);
        const double f = beta * (v0 * a0 + v1 * a1 + v2 * a2);
        at(H, ld, k, c) = a0 - f * v0;
        at(H, ld, k + 1, c) = a1 - f * v1;
        at(H, ld, k + 2, c) = a2 - f * v2;
      }
      __syncthreads();
      // right: columns k..k+2, rows lo..min(k+3, hi)
      const int r1 = min(k + 3, hi);
      for (int r = lo + lane; r <= r1; r += kWave) {
        const double a0 = at(H, ld, r, k), a1 = at(H, ld, r, k + 1),
                     a2 = at(H, ld, r, k + 2);
        const double f = beta * (a0 * v0 + a1 * v1 + a2 * v2);
        at(H, ld, r, k) = a0 - f * v0;
        at(H, ld, r, k + 1) = a1 - f * v1;
        at(H, ld, r, k + 2) = a2 - f * v2;
      }
      __syncthreads();
      x = at(H, ld, k + 1, k);
      y = at(H, ld, k + 2, k);
      z = k < hi - 2 ? at(H, ld, k + 3, k) : 0.0;
    }
    // final 2x2 reflector on rows hi-1..hi
    {
      const double nrm = sqrt(x * x + y * y);
      double v0 = 1.0, v1 = 0.0, beta = 0.0;
      if (nrm != 0.0) {
        const double alpha = x >= 0.0 ? -nrm : nrm;
        v0 = x - alpha;
        v1 = y;
        const double vv = v0 * v0 + v1 * v1;
        beta = vv > 0.0 ? 2.0 / vv : 0.0;
      }
      const int k = hi - 1;
      __syncthreads();
      for (int c = (k - 1 >= lo ? k - 1 : lo) + lane; c <= hi; c += kWave) {
        const double a0 = at(H, ld, k, c), a1 = at(H, ld, k + 1, c);
        const double f = beta * (v0 * a0 + v1 * a1);
        at(H, ld, k, c) = a0 - f * v0;
        at(H, ld, k + 1, c) = a1 - f * v1;
      }
      __syncthreads();
      for (int r = lo + lane; r <= hi; r += kWave) {
        const double a0 = at(H, ld, r, k), a1 = at(H, ld, r, k + 1);
        const double f = beta * (a0 * v0 + a1 * v1);
        at(H, ld, r, k) = a0 - f * v0;
        at(H, ld, r, k + 1) = a1 - f * v1;
      }
      __syncthreads();
    }
  }
  if (lane == 0) *status = ok ? 0 : 1;
}

// One wavefront; the window lives in LDS up to order 128 (body instantiated
// with the LDS array so its accesses compile to ds_* instructions), in
// global scratch above.
__global__ __launch_bounds__(kWave) void k_hqr(const double* __restrict__ Hin,
                                               int ldh, int n, double* wr,
                                               double* wi, double* scratch,
                                               int* status) {
  // odd leading dimension: a row of the window spreads over the LDS banks
  __shared__ double Hs[(kHqrMax + 1) * kHqrMax];
  if (n <= kHqrMax)
    hqr_body(Hs, kHqrMax + 1, Hin, ldh, n, wr, wi, status);
  else
    hqr_body(scratch, n, Hin, ldh, n, wr, wi, status);
}

// ------------------------------------------------------------------ Leja
constexpr int kLejaBlock = 256;
constexpr int kLejaMax = 1024;

__device__ bool key_less(double ar, double ai, int a, double br, double bi,
                         int b) {
  // sort key: real part descending, imaginary part descending, index
  if (ar != br) return ar > br;
  if (ai != bi) return ai > bi;
  return a < b;
}

// Modified Leja order of the Ritz values, recurrence records and estimator.
// info_out: [0] s0* (0 when not computed), [1] gamma guard hits,
//           [2] status (0 ok, 1 non-finite values).
__global__ __launch_bounds__(kLejaBlock) void k_leja(
    const double* __restrict__ wr_in, const double* __restrict__ wi_in,
    int m, int basis, double eps, double omega_est, double* ritz_out,
    double* rec, int* info_out, double* scratch) {
  __shared__ double sr[kLejaMax], si[kLejaMax], score[kLejaMax];
  __shared__ double lr_r[kLejaMax], lr_i[kLejaMax], gam[kLejaMax];
  __shared__ int taken[kLejaMax], zero[kLejaMax];
  __shared__ double red_v[kLejaBlock];
  __shared__ int red_i[kLejaBlock];
  __shared__ int pick;
  __shared__ double meanr, meani;
  const int tid = threadIdx.x;
  // 1. sort by (re desc, im desc, index)
  for (int k = tid; k < m; k += kLejaBlock) {
    const double ar = wr_in[k], ai = wi_in[k];
    int rank = 0;
    for (int q = 0; q < m; ++q)
      if (key_less(wr_in[q], wi_in[q], q, ar, ai, k)) ++rank;
    sr[rank] = ar;
    si[rank] = ai;
  }
  __syncthreads();
  for (int k = tid; k < m; k += kLejaBlock) {
    taken[k] = 0;
    zero[k] = 0;
    score[k] = 0.0;
  }
  __syncthreads();
  int bad = 0;
  for (int k = 0; k < m; ++k)
    if (!isfinite(sr[k]) || !isfinite(si[k])) bad = 1;
  // 2. greedy selection
  auto take = [&](int k, int pos) {
    if (tid == 0) {
      lr_r[pos] = sr[k];
      lr_i[pos] = si[k];
      taken[k] = 1;
    }
    __syncthreads();
    for (int q = tid; q < m; q += kLejaBlock) {
      if (taken[q]) continue;
      const double d = hypot(sr[q] - sr[k], si[q] - si[k]);
      if (d == 0.0) zero[q] = 1;
      else score[q] += log(d);
    }
    __syncthreads();
  };
  // first: largest modulus, earliest in sorted order among near-ties
  if (tid == 0) {
    double best = 0.0;
    for (int k = 0; k < m; ++k) best = fmax(best, hypot(sr[k], si[k]));
    int f = 0;
    for (int k = 0; k < m; ++k)
      if (hypot(sr[k], si[k]) >= best * (1.0 - 1e-15)) { f = k; break; }
    pick = f;
  }
  __syncthreads();
  int pos = 0;
  while (pos < m) {
    const int k = pick;
    take(k, pos++);
    if (si[k] != 0.0 && pos < m) {
      if (tid == 0) {
        int c = -1;
        for (int q = 0; q < m; ++q)
          if (!taken[q] && sr[q] == sr[k] && si[q] == -si[k]) { c = q; break; }
        pick = c;
      }
      __syncthreads();
      if (pick < 0) { bad = 1; break; }
      take(pick, pos++);
    }
    if (pos >= m) break;
    // next: maximal score; near-ties go to the earliest in sorted order
    double bv = -INFINITY;
    for (int q = tid; q < m; q += kLejaBlock)
      if (!taken[q] && !zero[q] && score[q] > bv) bv = score[q];
    red_v[tid] = bv;
    __syncthreads();
    if (tid == 0) {
      double top = -INFINITY;
      for (int i = 0; i < kLejaBlock; ++i) top = fmax(top, red_v[i]);
      int f = -1;
      if (top == -INFINITY) {
        for (int q = 0; q < m; ++q)
          if (!taken[q]) { f = q; break; }
      } else {
        const double tolv = 1e-10 * fmax(1.0, fabs(top));
        for (int q = 0; q < m; ++q)
          if (!taken[q] && !zero[q] && score[q] >= top - tolv) { f = q; break; }
      }
      pick = f;
    }
    __syncthreads();
  }
  // 3. mean, gamma, records (in Leja order: lr_r / lr_i)
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < m; ++k) { a += lr_r[k]; b += lr_i[k]; }
    meanr = a / m;
    meani = b / m;
  }
  __syncthreads();
  for (int k = tid; k < m; k += kLejaBlock)
    gam[k] = basis == SGM_BASIS_SCALED_NEWTON
                 ? hypot(meanr - lr_r[k], meani - lr_i[k])
                 : 1.0;
  __syncthreads();
  int hits = 0;
  if (basis == SGM_BASIS_SCALED_NEWTON) {
    double gmax = 0.0;
    for (int k = 0; k < m; ++k) gmax = fmax(gmax, gam[k]);
    const double floor_v = gmax > 0.0 ? 1e-12 * gmax : 1.0;
    for (int k = 0; k < m; ++k) hits += gam[k] < floor_v;
    __syncthreads();
    for (int k = tid; k < m; k += kLejaBlock) gam[k] = fmax(gam[k], floor_v);
    __syncthreads();
  }
  if (tid == 0) {
    int j = 0;
    while (j < m) {
      rec[3 * j] = lr_r[j];
      rec[3 * j + 1] = gam[j];
      rec[3 * j + 2] = 0.0;
      if (lr_i[j] != 0.0 && j + 1 < m) {
        const double be = fabs(lr_i[j]);
        rec[3 * (j + 1)] = lr_r[j + 1];
        rec[3 * (j + 1) + 1] = gam[j + 1];
        rec[3 * (j + 1) + 2] = -be * be / gam[j];
        j += 2;
      } else {
        j += 1;
      }
    }
    for (int k = 0; k < m; ++k) {
      ritz_out[2 * k] = lr_r[k];
      ritz_out[2 * k + 1] = lr_i[k];
    }
  }
  __syncthreads();
  // 4. estimator: log E (row i by thread i), column 2-norms
  int s0 = 0;
  if (basis == SGM_BASIS_SCALED_NEWTON && omega_est > 0.0) {
    double* L = scratch;  // m x m, L[j * m + i]
    const double leps = log(eps);
    for (int i = tid; i < m; i += kLejaBlock) {
      double acc = 0.0;
      for (int j = 0; j < m; ++j) {
        const double lrij =
            log(hypot(lr_r[i] - lr_r[j], lr_i[i] - lr_i[j])) - log(gam[j]);
        if (j < i) {
          L[(int64_t)j * m + i] = acc;
          acc += lrij;
        } else if (j == i) {
          acc += leps;
          L[(int64_t)j * m + i] = acc;
        } else {
          L[(int64_t)j * m + i] = acc;
          acc += lrij;
        }
      }
    }
    __syncthreads();
    double* nrm = scratch + (int64_t)m * m;
    for (int j = tid; j < m; j += kLejaBlock) {
      const double* col = L + (int64_t)j * m;
      double mx = -INFINITY;
      for (int i = 0; i < m; ++i) mx = fmax(mx, col[i]);
      if (mx == -INFINITY) {
        nrm[j] = -INFINITY;
      } else {
        double sm = 0.0;
        for (int i = 0; i < m; ++i) sm += exp(2.0 * (col[i] - mx));
        nrm[j] = mx + 0.5 * log(sm);
      }
    }
    __syncthreads();
    if (tid == 0) {
      const double lo = log(omega_est);
      int f = m;
      for (int j = 0; j < m; ++j)
        if (nrm[j] >= lo) { f = j; break; }
      s0 = f < 1 ? 1 : f;
    }
  }
  if (tid == 0) {
    info_out[0] = s0;
    info_out[1] = hits;
    info_out[2] = bad;
  }
}

}  // namespace

void hqr_eigen(const double* H, int ldh, int m0, double* wr, double* wi,
               double* scratch, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_hqr, dim3(1), dim3(kWave), 0, st, H, ldh, m0, wr, wi,
                     scratch, status);
  SGM_CHECK_LAUNCH();
}

size_t shifts_scratch_doubles(int m0) {
  return (size_t)m0 * m0 + (size_t)m0 + 16;
}

void leja_records(const double* wr, const double* wi, int m0, int basis,
                  double eps, double omega_est, double* ritz_out, double* rec,
                  int* info_out, double* scratch, hipStream_t st) {
  if (m0 > kLejaMax) throw Error{SGM_EINVAL, "more than 1024 Ritz values"};
  hipLaunchKernelGGL(k_leja, dim3(1), dim3(kLejaBlock), 0, st, wr, wi, m0,
                     basis, eps, omega_est, ritz_out, rec, info_out, scratch);
  SGM_CHECK_LAUNCH();
}

}  // namespace sgm
