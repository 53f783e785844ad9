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
// eigenvalues are needed.  One wavefront; scalars are computed redundantly
// by every lane.
//
// The matrix is stored packed, column c holding rows 0..c+1 (the Hessenberg
// part only): entries that a chase step annihilates are set to zero rather
// than stored, and the three bulge entries below the subdiagonal never
// reach memory.  Each chase step k applies its reflector from the left to
// rows k..k+2 and from the right to columns k..k+2, but the right-hand
// update of rows k..k+3 is deferred to step k+1: every lane carries that
// 4 x 3 block (post left update) in registers and finishes it there, which
// also yields the next reflector's vector (x, y, z) without a round trip
// through memory.  What a step writes is then never read by another lane
// in the same step, so one barrier per chase step suffices.  The result is
// the textbook iteration with the annihilated entries set to exact zeros.
constexpr int kHqrLdsOrder = 200;  // packed window in LDS up to this order
constexpr int kHqrLdsDoubles = (kHqrLdsOrder * (kHqrLdsOrder + 3) - 2) / 2;

// offset of column c in the packed storage
__device__ __forceinline__ int hcol(int c) { return c * (c + 3) / 2; }

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

// a -= beta (v . a) v for a 3-vector (a reflector applied from the left)
__device__ __forceinline__ void refl3_left(double& a0, double& a1, double& a2,
                                           double v0, double v1, double v2,
                                           double beta) {
  const double f = beta * (v0 * a0 + v1 * a1 + v2 * a2);
  a0 = a0 - f * v0;
  a1 = a1 - f * v1;
  a2 = a2 - f * v2;
}

// the same applied to a row from the right
__device__ __forceinline__ void refl3_right(double& a0, double& a1, double& a2,
                                            double v0, double v1, double v2,
                                            double beta) {
  const double f = beta * (a0 * v0 + a1 * v1 + a2 * v2);
  a0 = a0 - f * v0;
  a1 = a1 - f * v1;
  a2 = a2 - f * v2;
}

// NQ: chunks of 64 lanes covering n (n <= 64 NQ).  H: packed storage of
// at least (n (n + 3) - 2) / 2 doubles.
template <int NQ>
__device__ __forceinline__ void hqr_body(double* H,
                                         const double* __restrict__ Hin,
                                         int ldh, int n, double* wr,
                                         double* wi, int* status) {
  const int lane = threadIdx.x;
  // copy in (16 loads in flight per lane), summing |h| for the deflation
  // test's fallback scale
  double part = 0.0;
  const int total_e = n * n;
  for (int e0 = 0; e0 < total_e; e0 += kWave * 16) {
    double t[16];
    int dst[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + lane + kWave * u;
      const int r = e % n, c = e / n;
      const bool in = e < total_e && r <= c + 1;
      dst[u] = in ? hcol(c) + r : -1;
      t[u] = in ? Hin[(int64_t)c * ldh + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (dst[u] >= 0) {
        H[dst[u]] = t[u];
        part += fabs(t[u]);
      }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
  const double anorm = part;
  __syncthreads();
  const double ulp = 2.220446049250313e-16;
  int hi = n - 1;
  int its = 0, total = 0;
  int ok = 1;
  while (hi >= 0) {
    // deflation: the largest r <= hi with a negligible H(r, r-1) starts the
    // unreduced window (0 if none); every lane tests one r per chunk
    int lo = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = hi - lane - kWave * q;
      bool neg = false;
      if (r >= 1) {
        double sc = fabs(H[hcol(r - 1) + r - 1]) + fabs(H[hcol(r) + r]);
        if (sc == 0.0) sc = anorm;
        neg = fabs(H[hcol(r - 1) + r]) <= ulp * sc;
      }
      const unsigned long long m = __ballot(neg);
      if (m != 0ull) {
        lo = hi - (kWave * q + __builtin_ctzll(m));
        break;
      }
    }
    if (lo > 0 && lane == 0) H[hcol(lo - 1) + lo] = 0.0;
    __syncthreads();
    if (lo == hi) {
      if (lane == 0) { wr[hi] = H[hcol(hi) + hi]; wi[hi] = 0.0; }
      hi -= 1;
      its = 0;
      continue;
    }
    if (lo == hi - 1) {
      double r1, i1, r2, i2;
      eig2(H[hcol(hi - 1) + hi - 1], H[hcol(hi) + hi - 1],
           H[hcol(hi - 1) + hi], H[hcol(hi) + hi], r1, i1, r2, i2);
      if (lane == 0) {
        wr[hi - 1] = r1; wi[hi - 1] = i1;
        wr[hi] = r2; wi[hi] = i2;
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > 40 * n) { ok = 0; break; }
    ++its;
    // shifts: eigenvalues of the trailing 2x2 (sum s, product t), or an
    // exceptional pair after 10 and 20 stagnant steps
    double s, t;
    const double hmm = H[hcol(hi - 1) + hi - 1], hnn = H[hcol(hi) + hi];
    if (its == 10 || its == 20) {
      const double w = fabs(H[hcol(hi - 1) + hi]) +
                       fabs(H[hcol(hi - 2) + hi - 1]);
      const double sh = hnn + 0.75 * w;
      s = 2.0 * sh;
      t = sh * sh + 0.25 * w * w;
    } else {
      s = hmm + hnn;
      t = hmm * hnn - H[hcol(hi) + hi - 1] * H[hcol(hi - 1) + hi];
    }
    const double l00 = H[hcol(lo) + lo], l10 = H[hcol(lo) + lo + 1];
    const double l01 = H[hcol(lo + 1) + lo], l11 = H[hcol(lo + 1) + lo + 1];
    const double l21 = H[hcol(lo + 1) + lo + 2];
    double x = l00 * l00 + l01 * l10 - s * l00 + t;
    double y = l10 * (l00 + l11 - s);
    double z = l10 * l21;
    // the pending block: rows k-1..k+2 of columns k-1..k+1 after the left
    // update of step k-1, before its right update; (pv, pb) its reflector
    double P[4][3];
    double pv0 = 0.0, pv1 = 0.0, pv2 = 0.0, pb = 0.0;
    for (int k = lo; k <= hi - 2; ++k) {
      const int b0 = hcol(k), b1 = hcol(k + 1), b2 = hcol(k + 2);
      // loads first: none depends on this step's reflector
      double a[NQ][3];  // rows k..k+2 of columns k+3+lane+64q
      double w3[NQ][3]; // columns k..k+2 of rows lo+lane+64q (< k)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = k + 3 + lane + kWave * q;
        if (c <= hi) {
          const int bc = hcol(c) + k;
          a[q][0] = H[bc]; a[q][1] = H[bc + 1]; a[q][2] = H[bc + 2];
        }
        const int r = lo + lane + kWave * q;
        if (r < k) {
          w3[q][0] = H[b0 + r]; w3[q][1] = H[b1 + r]; w3[q][2] = H[b2 + r];
        }
      }
      double S[3][3];  // rows k..k+2 of columns k..k+2 after the left update
      S[0][2] = H[b2 + k];
      S[1][2] = H[b2 + k + 1];
      S[2][2] = H[b2 + k + 2];
      double Pp[4][3];
      if (k > lo) {
        P[3][2] = H[b1 + k + 2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          Pp[i][0] = P[i][0]; Pp[i][1] = P[i][1]; Pp[i][2] = P[i][2];
          refl3_right(Pp[i][0], Pp[i][1], Pp[i][2], pv0, pv1, pv2, pb);
        }
        x = Pp[1][0];
        y = Pp[2][0];
        z = Pp[3][0];
      } else {
        S[0][0] = H[b0 + k]; S[1][0] = H[b0 + k + 1]; S[2][0] = 0.0;
        S[0][1] = H[b1 + k]; S[1][1] = H[b1 + k + 1]; S[2][1] = H[b1 + k + 2];
      }
      double v0, v1, v2, beta;
      house3(x, y, z, v0, v1, v2, beta);
      if (k > lo) {
        // column k-1: row k-1 is final, row k gets the left update, rows
        // k+1 and k+2 are annihilated
        double t0 = Pp[1][0], t1 = Pp[2][0], t2 = Pp[3][0];
        refl3_left(t0, t1, t2, v0, v1, v2, beta);
        if (lane == 0) {
          const int bm = hcol(k - 1);
          H[bm + k - 1] = Pp[0][0];
          H[bm + k] = t0;
        }
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          S[0][d] = Pp[1][d + 1];
          S[1][d] = Pp[2][d + 1];
          S[2][d] = Pp[3][d + 1];
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
        refl3_left(S[0][d], S[1][d], S[2][d], v0, v1, v2, beta);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = k + 3 + lane + kWave * q;
        if (c <= hi) {
          refl3_left(a[q][0], a[q][1], a[q][2], v0, v1, v2, beta);
          const int bc = hcol(c) + k;
          H[bc] = a[q][0]; H[bc + 1] = a[q][1]; H[bc + 2] = a[q][2];
        }
        const int r = lo + lane + kWave * q;
        if (r < k) {
          double c0 = w3[q][0], c1 = w3[q][1];
          if (r == k - 1) { c0 = Pp[0][1]; c1 = Pp[0][2]; }
          double c2 = w3[q][2];
          refl3_right(c0, c1, c2, v0, v1, v2, beta);
          H[b0 + r] = c0; H[b1 + r] = c1; H[b2 + r] = c2;
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        P[0][d] = S[0][d]; P[1][d] = S[1][d]; P[2][d] = S[2][d];
      }
      P[3][0] = 0.0;
      P[3][1] = 0.0;
      pv0 = v0; pv1 = v1; pv2 = v2; pb = beta;
      __syncthreads();
    }
    // final 2x2 reflector on rows / columns hi-1..hi, after the pending
    // right update of step hi-2 on rows hi-2..hi
    {
      const int bh1 = hcol(hi - 1), bh = hcol(hi);
      double w2[NQ][2];  // columns hi-1, hi of rows lo+lane+64q (< hi-2)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = lo + lane + kWave * q;
        if (r < hi - 2) { w2[q][0] = H[bh1 + r]; w2[q][1] = H[bh + r]; }
      }
      double Pp[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Pp[i][0] = P[i][0]; Pp[i][1] = P[i][1]; Pp[i][2] = P[i][2];
        refl3_right(Pp[i][0], Pp[i][1], Pp[i][2], pv0, pv1, pv2, pb);
      }
      x = Pp[1][0];
      y = Pp[2][0];
      const double nrm = sqrt(x * x + y * y);
      double v0 = 1.0, v1 = 0.0, beta = 0.0;
      if (nrm != 0.0) {
        const double alpha = x >= 0.0 ? -nrm : nrm;
        v0 = x - alpha;
        v1 = y;
        const double vv = v0 * v0 + v1 * v1;
        beta = vv > 0.0 ? 2.0 / vv : 0.0;
      }
      // left update of columns hi-2..hi (rows hi-1, hi); L[d][i]: column
      // hi-2+d, row hi-1+i
      double L[3][2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double a0 = Pp[1][d], a1 = Pp[2][d];
        const double f = beta * (v0 * a0 + v1 * a1);
        L[d][0] = a0 - f * v0;
        L[d][1] = a1 - f * v1;
      }
      if (lane == 0) {
        const int bm = hcol(hi - 2);
        H[bm + hi - 2] = Pp[0][0];
        H[bm + hi - 1] = L[0][0];
      }
      // right update of columns hi-1, hi for rows lo..hi
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = lo + lane + kWave * q;
        if (r <= hi) {
          double a0, a1;
          if (r < hi - 2) { a0 = w2[q][0]; a1 = w2[q][1]; }
          else if (r == hi - 2) { a0 = Pp[0][1]; a1 = Pp[0][2]; }
          else if (r == hi - 1) { a0 = L[1][0]; a1 = L[2][0]; }
          else { a0 = L[1][1]; a1 = L[2][1]; }
          const double f = beta * (a0 * v0 + a1 * v1);
          H[bh1 + r] = a0 - f * v0;
          H[bh + r] = a1 - f * v1;
        }
      }
      __syncthreads();
    }
  }
  if (lane == 0) *status = ok ? 0 : 1;
}

// One wavefront; the packed window lives in LDS up to order 200 (the body
// instantiated with the LDS array so its accesses compile to ds_*
// instructions), in global scratch above.
template <int NQ>
__global__ __launch_bounds__(kWave) void k_hqr(const double* __restrict__ Hin,
                                               int ldh, int n, double* wr,
                                               double* wi, double* scratch,
                                               int* status) {
  if constexpr (NQ * kWave <= 256) {
    __shared__ double Hs[kHqrLdsDoubles];
    if (n <= kHqrLdsOrder) {
      hqr_body<NQ>(Hs, Hin, ldh, n, wr, wi, status);
      return;
    }
  }
  hqr_body<NQ>(scratch, Hin, ldh, n, wr, wi, status);
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
  // scratch (used above order 200) holds m0 * m0 >= (m0 (m0 + 3) - 2) / 2
  // doubles
  if (m0 < 1 || m0 > 16 * kWave) throw Error{SGM_EINVAL, "hqr: order out of range"};
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(1), dim3(kWave), 0, st, H, ldh, m0, wr, wi,
                       scratch, status);
  };
  if (m0 <= kWave) go(k_hqr<1>);
  else if (m0 <= 2 * kWave) go(k_hqr<2>);
  else if (m0 <= 4 * kWave) go(k_hqr<4>);
  else if (m0 <= 8 * kWave) go(k_hqr<8>);
  else go(k_hqr<16>);
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
