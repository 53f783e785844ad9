// ILU(0) right preconditioning (the preconditioner of the 2D Laplace test
// with an ILU preconditioner, Sec. 4.3): the factorisation M = L U with zero
// fill-in and the two triangular solves M^{-1} r = U^{-1} (L^{-1} r), all on
// the GPU.
//
// Both substitutions are scheduled by level: the level of a row in the
// forward (backward) substitution is one more than the highest level among
// the rows of its strict lower (upper) part, so the rows of one level are
// independent.  One workgroup of 1024 threads walks the levels in order with
// a barrier between them; the y values it reads were written by the same
// workgroup before the barrier.  The solves are bound by that chain of
// levels (about 2 N for an N x N 5-point grid in natural order), not by
// bandwidth: a dependent global round trip per level.
//
// Within a level the rows are sorted, and each row's strict triangle is
// stored per position in level order (ELL: entry t of position p at
// t * n + p), so a level's threads read consecutive addresses.
#include "internal.h"

#include <hipcub/hipcub.hpp>

namespace sgm {

namespace {

constexpr int kIluBlock = 1024;
constexpr int kLevDeps = 8;  // dependencies a row keeps in registers

__global__ void k_ilu_check(const int32_t* rp, const int32_t* col, int64_t n,
                            int32_t* dpos, int32_t* flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t d = -1;
  bool sorted = true;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
    if (col[e] == i) d = e;
    if (e > rp[i] && col[e] <= col[e - 1]) sorted = false;
  }
  dpos[i] = d;
  if (d < 0) flags[0] = 1;        // missing diagonal
  if (!sorted) flags[1] = 1;      // unsorted (or duplicate) columns
}

// Entries of row i on the strict lower (upper = 0) or strict upper
// (upper = 1) side of the diagonal: CSR range [e0, e1).
__device__ __forceinline__ void tri_range(const int32_t* rp,
                                          const int32_t* dpos, int64_t i,
                                          int upper, int32_t& e0,
                                          int32_t& e1) {
  if (upper) {
    e0 = dpos[i] + 1;
    e1 = rp[i + 1];
  } else {
    e0 = rp[i];
    e1 = dpos[i];
  }
}

// Levels of one substitution (upper = 0 forward, 1 backward) and their
// count.  One wavefront visits the rows in dependency order (increasing for
// the forward, decreasing for the backward substitution), 64 at a time.
// Dependencies on earlier batches are final; those inside the batch are
// resolved by repeating the batch's update until nothing changes, which
// takes at most 64 passes (no dependency chain inside a batch is longer).
// A row keeps up to kLevDeps in-batch dependencies in registers and reads
// any others again each pass.
__global__ __launch_bounds__(kWave) void k_ilu_levels(
    const int32_t* rp, const int32_t* col, const int32_t* dpos, int64_t n,
    int upper, int32_t* lev, int32_t* nlev, int32_t* width) {
  __shared__ int32_t sl[kWave];
  const int lane = threadIdx.x;
  int32_t top = -1, wmax = 0;
  for (int64_t b0 = 0; b0 < n; b0 += kWave) {
    const int64_t q = b0 + lane;  // position in dependency order
    const bool ok = q < n;
    const int64_t i = upper ? n - 1 - q : q;
    int32_t e0 = 0, e1 = 0;
    if (ok) tri_range(rp, dpos, i, upper, e0, e1);
    wmax = max(wmax, e1 - e0);
    int32_t ext = -1;
    int dep[kLevDeps];
    int nd = 0;
    bool more = false;
    for (int32_t e = e0; e < e1; ++e) {
      const int64_t k = col[e];
      const int64_t qk = upper ? n - 1 - k : k;
      if (qk < b0) {
        ext = max(ext, lev[k]);
      } else if (nd < kLevDeps) {
        dep[nd++] = (int)(qk - b0);
      } else {
        more = true;
      }
    }
    int32_t my = ext + 1;
    for (int pass = 0; pass <= kWave; ++pass) {
      sl[lane] = my;
      __syncthreads();
      int32_t nw = ext + 1;
#pragma unroll
      for (int u = 0; u < kLevDeps; ++u)
        if (u < nd) nw = max(nw, sl[dep[u]] + 1);
      if (more) {
        for (int32_t e = e0; e < e1; ++e) {
          const int64_t k = col[e];
          const int64_t qk = upper ? n - 1 - k : k;
          if (qk >= b0) nw = max(nw, sl[qk - b0] + 1);
        }
      }
      __syncthreads();
      const bool changed = __any(nw != my);
      my = nw;
      if (!changed) break;
    }
    if (ok) {
      lev[i] = my;
      top = max(top, my);
    }
    __syncthreads();
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    top = max(top, __shfl_xor(top, off));
    wmax = max(wmax, __shfl_xor(wmax, off));
  }
  if (lane == 0) {
    nlev[0] = top + 1;
    width[0] = wmax;
  }
}

__global__ void k_iota32(int32_t* a, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

// ptr[l] = first position of level l in the sorted order, ptr[nlev] = n
// (every level 0 .. nlev - 1 holds at least one row).
__global__ void k_level_starts(const int32_t* key, int64_t n, int32_t* ptr,
                               const int32_t* nlev) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (p == 0 || key[p] != key[p - 1]) ptr[key[p]] = (int32_t)p;
  if (p == n - 1) ptr[nlev[0]] = (int32_t)n;
}

// The strict triangle of each position's row in level order (ELL).
__global__ void k_ilu_ell(const int32_t* rp, const int32_t* col,
                          const int32_t* dpos, const int32_t* rows,
                          int64_t n, int upper, int32_t width, int32_t* cnt,
                          int32_t* ecol, int32_t* esrc) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t i = rows[p];
  int32_t e0, e1;
  tri_range(rp, dpos, i, upper, e0, e1);
  cnt[p] = e1 - e0;
  for (int32_t t = 0; t < width; ++t) {
    const bool in = t < e1 - e0;
    ecol[(int64_t)t * n + p] = in ? col[e0 + t] : 0;
    esrc[(int64_t)t * n + p] = in ? e0 + t : -1;
  }
}

// ILU(0) in the IKJ form on the forward-substitution levels: row i is
// eliminated with its lower entries k in increasing order (rows k are
// final, they sit on earlier levels): l_ik = a_ik / u_kk, then
// a_ij -= l_ik u_kj for the entries j > k of row k that row i also holds
// (a merge of the two sorted column lists); fill outside the pattern is
// dropped.  f holds A's values on entry and L (strict lower) and U on exit,
// in A's CSR order.  bad[0] is set on a zero or non-finite pivot.
__global__ __launch_bounds__(kIluBlock) void k_ilu_factor(
    const int32_t* rp, const int32_t* col, const int32_t* dpos,
    const int32_t* rows, const int32_t* lptr, const int32_t* nlev, double* f,
    int32_t* bad) {
  const int nl = nlev[0];
  bool flag = false;
  for (int l = 0; l < nl; ++l) {
    const int p1 = lptr[l + 1];
    for (int p = lptr[l] + (int)threadIdx.x; p < p1; p += kIluBlock) {
      const int i = rows[p];
      const int end = rp[i + 1];
      const int di = dpos[i];
      for (int e = rp[i]; e < di; ++e) {
        const int k = col[e];
        const double piv = f[dpos[k]];
        if (!(piv != 0.0 && isfinite(piv))) flag = true;
        const double lik = f[e] / piv;
        f[e] = lik;
        int t = e + 1, g = dpos[k] + 1;
        const int gend = rp[k + 1];
        while (t < end && g < gend) {
          const int ct = col[t], cg = col[g];
          if (ct == cg) {
            f[t] -= lik * f[g];
            ++t;
            ++g;
          } else if (ct < cg) {
            ++t;
          } else {
            ++g;
          }
        }
      }
      const double d = f[di];
      if (!(d != 0.0 && isfinite(d))) flag = true;
    }
    __syncthreads();
  }
  if (flag) bad[0] = 1;
}

// Factor values per ELL position, and 1 / u_ii for the backward levels.
__global__ void k_ilu_ell_vals(const int32_t* esrc, const int32_t* cnt,
                               int64_t n, int32_t width, const double* f,
                               double* eval) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int c = cnt[p];
  for (int t = 0; t < width; ++t) {
    const int64_t q = (int64_t)t * n + p;
    eval[q] = t < c ? f[esrc[q]] : 0.0;
  }
}

__global__ void k_ilu_dinv(const int32_t* rows, const int32_t* dpos,
                           int64_t n, const double* f, double* dinv) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) dinv[p] = 1.0 / f[dpos[rows[p]]];
}

struct IluSide {
  const int32_t* rows;
  const int32_t* lptr;
  const int32_t* cnt;
  const int32_t* ecol;
  const double* eval;
};

// z = M^{-1} b: the forward substitution L y = b over its levels, then the
// backward substitution U z = y over its levels, in place in z.  b is read
// at BV.row_off(row) (a basis column or a plain vector; it may be z itself).
__global__ __launch_bounds__(kIluBlock) void k_ilu_apply(
    QView<const double> BV, const double* b, double* z, IluSide L, IluSide U,
    const double* __restrict__ dinv, const int32_t* __restrict__ nlev,
    int64_t n) {
  const int nl = nlev[0], nu = nlev[1];
  for (int l = 0; l < nl; ++l) {
    const int p1 = L.lptr[l + 1];
    for (int p = L.lptr[l] + (int)threadIdx.x; p < p1; p += kIluBlock) {
      const int r = L.rows[p];
      double s = b[BV.row_off(r)];
      const int c = L.cnt[p];
      for (int t = 0; t < c; ++t) {
        const int64_t q = (int64_t)t * n + p;
        s -= L.eval[q] * z[L.ecol[q]];
      }
      z[r] = s;
    }
    __syncthreads();
  }
  for (int l = 0; l < nu; ++l) {
    const int p1 = U.lptr[l + 1];
    for (int p = U.lptr[l] + (int)threadIdx.x; p < p1; p += kIluBlock) {
      const int r = U.rows[p];
      double s = z[r];
      const int c = U.cnt[p];
      for (int t = 0; t < c; ++t) {
        const int64_t q = (int64_t)t * n + p;
        s -= U.eval[q] * z[U.ecol[q]];
      }
      z[r] = s * dinv[p];
    }
    __syncthreads();
  }
}

inline unsigned g256(int64_t n) {
  return (unsigned)ceil_div(n > 0 ? n : 1, 256);
}

template <typename T>
T* dalloc(int64_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * (size_t)(count > 0 ? count : 1)) !=
      hipSuccess)
    throw Error{SGM_ENOMEM, "ILU(0): device allocation failed"};
  return static_cast<T*>(p);
}

// Levels, sorted rows, level starts and the ELL structure of one side.
void build_side(const Matrix& M, const int32_t* dpos, int upper,
                IluLevels& S, int32_t* nlev_dev, hipStream_t st) {
  const int64_t n = M.n;
  int32_t* lev = dalloc<int32_t>(n);
  int32_t* key = dalloc<int32_t>(n);
  int32_t* iota = dalloc<int32_t>(n);
  int32_t* wdev = dalloc<int32_t>(1);
  hipLaunchKernelGGL(k_ilu_levels, dim3(1), dim3(kWave), 0, st, M.row_ptr,
                     M.col, dpos, n, upper, lev, nlev_dev, wdev);
  SGM_CHECK_LAUNCH();
  int32_t h[2] = {0, 0};
  SGM_HIP(hipMemcpyAsync(&h[0], nlev_dev, sizeof(int32_t),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipMemcpyAsync(&h[1], wdev, sizeof(int32_t), hipMemcpyDeviceToHost,
                         st));
  SGM_HIP(hipStreamSynchronize(st));
  S.nlev = h[0];
  S.width = h[1];
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) <= S.nlev) ++bits;
  S.rows = dalloc<int32_t>(n);
  hipLaunchKernelGGL(k_iota32, dim3(g256(n)), dim3(256), 0, st, iota, n);
  SGM_CHECK_LAUNCH();
  size_t tb = 0;
  SGM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, lev, key, iota,
                                             S.rows, (int)n, 0, bits, st));
  void* tmp = dalloc<char>((int64_t)tb);
  SGM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, lev, key, iota, S.rows,
                                             (int)n, 0, bits, st));
  S.lptr = dalloc<int32_t>(S.nlev + 1);
  hipLaunchKernelGGL(k_level_starts, dim3(g256(n)), dim3(256), 0, st, key, n,
                     S.lptr, nlev_dev);
  SGM_CHECK_LAUNCH();
  const int64_t wn = (int64_t)(S.width > 0 ? S.width : 1) * n;
  S.cnt = dalloc<int32_t>(n);
  S.ecol = dalloc<int32_t>(wn);
  S.esrc = dalloc<int32_t>(wn);
  S.eval = dalloc<double>(wn);
  hipLaunchKernelGGL(k_ilu_ell, dim3(g256(n)), dim3(256), 0, st, M.row_ptr,
                     M.col, dpos, S.rows, n, upper, S.width, S.cnt, S.ecol,
                     S.esrc);
  SGM_CHECK_LAUNCH();
  SGM_HIP(hipStreamSynchronize(st));
  for (void* p : {(void*)lev, (void*)key, (void*)iota, (void*)wdev, tmp})
    (void)hipFree(p);
}

void free_side(IluLevels& S) {
  for (void* p : {(void*)S.rows, (void*)S.lptr, (void*)S.cnt,
                  (void*)S.ecol, (void*)S.esrc, (void*)S.eval})
    if (p) (void)hipFree(p);
  S = IluLevels{};
}

}  // namespace

void ilu_free(Ilu*& I) {
  if (!I) return;
  free_side(I->L);
  free_side(I->U);
  for (void* p : {(void*)I->dpos, (void*)I->fac, (void*)I->dinv,
                  (void*)I->nlev_dev, (void*)I->flags})
    if (p) (void)hipFree(p);
  delete I;
  I = nullptr;
}

void ilu_factor(Matrix& M, hipStream_t st) {
  Ilu& I = *M.ilu;
  const int64_t n = M.n;
  SGM_HIP(hipMemcpyAsync(I.fac, M.val, sizeof(double) * (size_t)M.nnz,
                         hipMemcpyDeviceToDevice, st));
  SGM_HIP(hipMemsetAsync(I.flags + 2, 0, sizeof(int32_t), st));
  hipLaunchKernelGGL(k_ilu_factor, dim3(1), dim3(kIluBlock), 0, st,
                     M.row_ptr, M.col, I.dpos, I.L.rows, I.L.lptr,
                     I.nlev_dev, I.fac, I.flags + 2);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ilu_ell_vals, dim3(g256(n)), dim3(256), 0, st,
                     I.L.esrc, I.L.cnt, n, I.L.width, I.fac, I.L.eval);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ilu_ell_vals, dim3(g256(n)), dim3(256), 0, st,
                     I.U.esrc, I.U.cnt, n, I.U.width, I.fac, I.U.eval);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ilu_dinv, dim3(g256(n)), dim3(256), 0, st, I.U.rows,
                     I.dpos, n, I.fac, I.dinv);
  SGM_CHECK_LAUNCH();
  int32_t bad = 0;
  SGM_HIP(hipMemcpyAsync(&bad, I.flags + 2, sizeof(int32_t),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipStreamSynchronize(st));
  I.ok = bad == 0;
  if (!I.ok)
    throw Error{SGM_ENUMERIC, "ILU(0): zero or non-finite pivot"};
}

void ilu_build(Matrix& M, hipStream_t st) {
  const int64_t n = M.n;
  if (n > INT32_MAX - 1)
    throw Error{SGM_EINVAL, "ILU(0): n must be below 2^31 - 1"};
  ilu_free(M.ilu);
  M.ilu = new Ilu();
  Ilu& I = *M.ilu;
  try {
    I.dpos = dalloc<int32_t>(n);
    I.flags = dalloc<int32_t>(4);
    I.nlev_dev = dalloc<int32_t>(2);
    I.fac = dalloc<double>(M.nnz);
    I.dinv = dalloc<double>(n);
    SGM_HIP(hipMemsetAsync(I.flags, 0, sizeof(int32_t) * 4, st));
    hipLaunchKernelGGL(k_ilu_check, dim3(g256(n)), dim3(256), 0, st,
                       M.row_ptr, M.col, n, I.dpos, I.flags);
    SGM_CHECK_LAUNCH();
    int32_t fl[2] = {0, 0};
    SGM_HIP(hipMemcpyAsync(fl, I.flags, sizeof(fl), hipMemcpyDeviceToHost,
                           st));
    SGM_HIP(hipStreamSynchronize(st));
    if (fl[0])
      throw Error{SGM_EINVAL, "ILU(0): every diagonal entry must be stored"};
    if (fl[1])
      throw Error{SGM_EINVAL,
                  "ILU(0): column indices must be sorted within each row"};
    build_side(M, I.dpos, 0, I.L, I.nlev_dev, st);
    build_side(M, I.dpos, 1, I.U, I.nlev_dev + 1, st);
    ilu_factor(M, st);
  } catch (...) {
    ilu_free(M.ilu);
    throw;
  }
}

void ilu_apply(const Ilu& I, int64_t n, QView<const double> BV,
               const double* b, double* z, hipStream_t st) {
  const IluSide L{I.L.rows, I.L.lptr, I.L.cnt, I.L.ecol, I.L.eval};
  const IluSide U{I.U.rows, I.U.lptr, I.U.cnt, I.U.ecol, I.U.eval};
  hipLaunchKernelGGL(k_ilu_apply, dim3(1), dim3(kIluBlock), 0, st, BV, b, z,
                     L, U, (const double*)I.dinv, (const int32_t*)I.nlev_dev,
                     n);
  SGM_CHECK_LAUNCH();
}

}  // namespace sgm
