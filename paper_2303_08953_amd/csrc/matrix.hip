// Matrix analysis on the GPU: CSR -> SELL-C (C = 64) for A and A^T, float32
// value copy, diagonal, and validation of the caller's CSR arrays.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace sgm {

namespace {

__global__ void k_validate(const int32_t* rp, const int32_t* col, int64_t n,
                           int64_t nnz, int* bad) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r > n) return;
  if (r == 0 && rp[0] != 0) atomicOr(bad, 1);
  if (r == n) {
    if (rp[n] != nnz) atomicOr(bad, 2);
    return;
  }
  int32_t a = rp[r], b = rp[r + 1];
  if (b < a || a < 0 || b > nnz) {
    atomicOr(bad, 4);
    return;
  }
  for (int32_t k = a; k < b; ++k) {
    int32_t c = col[k];
    if (c < 0 || c >= n) {
      atomicOr(bad, 8);
      return;
    }
  }
}

__global__ void k_row_of(const int32_t* rp, int64_t n, int32_t* row_of) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) row_of[k] = (int32_t)r;
}

__global__ void k_diag(const int32_t* rp, const int32_t* col,
                       const double* val, int64_t n, double* diag) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double d = 0.0;
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k)
    if (col[k] == r) d += val[k];
  diag[r] = d;
}

// One wavefront per slice: width = longest row of the slice.
__global__ void k_slice_width(const int32_t* rp, int64_t n, int64_t nslices,
                              int32_t* width, int64_t* sizes) {
  int64_t s = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x % kWave;
  if (s >= nslices) return;
  int64_t r = s * kSlice + lane;
  int len = r < n ? rp[r + 1] - rp[r] : 0;
  for (int off = kWave / 2; off > 0; off >>= 1)
    len = max(len, __shfl_xor(len, off));
  if (lane == 0) {
    width[s] = len;
    sizes[s] = (int64_t)len * kSlice;
  }
}

__global__ void k_sell_fill(const int32_t* rp, const int32_t* col,
                            const int32_t* perm, int64_t n, int64_t nslices,
                            const int64_t* ptr, const int32_t* width,
                            int32_t* scol, int64_t* ssrc) {
  int64_t s = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x % kWave;
  if (s >= nslices) return;
  int64_t r = s * kSlice + lane;
  int64_t base = ptr[s] + lane;
  int w = width[s];
  int32_t a = r < n ? rp[r] : 0;
  int32_t len = r < n ? rp[r + 1] - a : 0;
  int32_t padcol = len > 0 ? col[a + len - 1] : (int32_t)(r < n ? r : 0);
  for (int k = 0; k < w; ++k) {
    int64_t e = base + (int64_t)k * kSlice;
    if (k < len) {
      scol[e] = col[a + k];
      ssrc[e] = perm ? (int64_t)perm[a + k] : (int64_t)(a + k);
    } else {
      scol[e] = padcol;
      ssrc[e] = -1;
    }
  }
}

// Group bases of the 16-bit relative columns.  One wavefront per slice;
// for every position w < width[s], the group's (column - lane) values over
// the slice's real rows (lane 0 always is one) give lo and hi; the base is
// lo + ceil((hi - lo) / 2), so every offset lies in [-32768, 32767] exactly
// when hi - lo <= 65535.  out[0] = the largest hi - lo (integer max: the
// result does not depend on the order of the atomics).
__global__ void k_sell_bases(const int32_t* scol, const int64_t* ptr,
                             const int32_t* width, int64_t n, int64_t nslices,
                             int32_t* kbase, int32_t* out) {
  int64_t s = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x % kWave;
  if (s >= nslices) return;
  const int64_t r = s * kSlice + lane;
  const int64_t base = ptr[s] + lane;
  const int w = width[s];
  int64_t span = 0;
  for (int k = 0; k < w; ++k) {
    const int64_t v = (int64_t)scol[base + (int64_t)k * kSlice] - lane;
    int64_t lo = r < n ? v : INT64_MAX, hi = r < n ? v : INT64_MIN;
    for (int off = kWave / 2; off > 0; off >>= 1) {
      lo = min(lo, (int64_t)__shfl_xor((long long)lo, off));
      hi = max(hi, (int64_t)__shfl_xor((long long)hi, off));
    }
    if (lane == 0) kbase[(ptr[s] >> 6) + k] = (int32_t)(lo + (hi - lo + 1) / 2);
    span = max(span, hi - lo);
  }
  if (lane == 0) atomicMax(out, (int32_t)min(span, (int64_t)INT32_MAX));
}

// 16-bit offsets against the group bases; rows past n take the column
// base + lane clamped to [0, n) (value 0, a valid gather address).
__global__ void k_sell_rel16(const int32_t* scol, const int64_t* ptr,
                             const int32_t* width, const int32_t* kbase,
                             int64_t n, int64_t nslices, int16_t* rcol) {
  int64_t s = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x % kWave;
  if (s >= nslices) return;
  const int64_t r = s * kSlice + lane;
  const int64_t base = ptr[s] + lane;
  const int w = width[s];
  for (int k = 0; k < w; ++k) {
    const int64_t e = base + (int64_t)k * kSlice;
    const int64_t b = kbase[(ptr[s] >> 6) + k];
    int64_t c = b + lane;
    if (r < n) c = scol[e];
    else c = c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
    rcol[e] = (int16_t)(c - lane - b);
  }
}

__global__ void k_sell_values(const int64_t* src, int64_t m,
                              const double* val, double* v64, float* v32) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  int64_t k = src[e];
  double v = k >= 0 ? val[k] : 0.0;
  v64[e] = v;
  v32[e] = (float)v;
}

__global__ void k_iota(int32_t* a, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

__global__ void k_count(const int32_t* col, int64_t nnz, int32_t* cnt) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_gather_i32(const int32_t* src, const int32_t* idx,
                             int64_t m, int32_t* out) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) out[k] = src[idx[k]];
}

inline unsigned grid1(int64_t n, int b = 256) {
  return (unsigned)ceil_div(n > 0 ? n : 1, b);
}

template <typename T>
T* dmalloc(int64_t count) {
  void* p = nullptr;
  if (count <= 0) count = 1;
  if (hipMalloc(&p, sizeof(T) * (size_t)count) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{SGM_ENOMEM, "hipMalloc of " +
                                std::to_string(sizeof(T) * (size_t)count) +
                                " bytes failed"};
  }
  return static_cast<T*>(p);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

void sell_build(Sell& S, int64_t n, const int32_t* rp, const int32_t* col,
                const int32_t* perm, hipStream_t st) {
  S.n = n;
  S.nslices = ceil_div(n, kSlice);
  S.ptr = dmalloc<int64_t>(S.nslices + 1);
  S.width = dmalloc<int32_t>(S.nslices);
  int64_t* sizes = dmalloc<int64_t>(S.nslices + 1);
  const int wpb = 4;  // slices per 256-thread block
  hipLaunchKernelGGL(k_slice_width, dim3(grid1(S.nslices, wpb)),
                     dim3(wpb * kWave), 0, st, rp, n, S.nslices, S.width,
                     sizes);
  SGM_CHECK_LAUNCH();
  SGM_HIP(hipMemsetAsync(sizes + S.nslices, 0, sizeof(int64_t), st));
  size_t tmp_bytes = 0;
  SGM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, sizes, S.ptr,
                                           (int)(S.nslices + 1), st));
  char* tmp = dmalloc<char>((int64_t)tmp_bytes);
  SGM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, sizes, S.ptr,
                                           (int)(S.nslices + 1), st));
  int64_t total = 0;
  SGM_HIP(hipMemcpyAsync(&total, S.ptr + S.nslices, sizeof(int64_t),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipStreamSynchronize(st));
  dfree(tmp);
  dfree(sizes);
  S.nnz_padded = total;
  S.col = dmalloc<int32_t>(total);
  S.src = dmalloc<int64_t>(total);
  S.val64 = dmalloc<double>(total);
  S.val32 = dmalloc<float>(total);
  hipLaunchKernelGGL(k_sell_fill, dim3(grid1(S.nslices, wpb)),
                     dim3(wpb * kWave), 0, st, rp, col, perm, n, S.nslices,
                     S.ptr, S.width, S.col, S.src);
  SGM_CHECK_LAUNCH();
  // 16-bit relative columns when every group's column range fits
  S.kbase = dmalloc<int32_t>(total / kSlice);
  int32_t* dspan = dmalloc<int32_t>(1);
  SGM_HIP(hipMemsetAsync(dspan, 0, sizeof(int32_t), st));
  hipLaunchKernelGGL(k_sell_bases, dim3(grid1(S.nslices, wpb)),
                     dim3(wpb * kWave), 0, st, S.col, S.ptr, S.width, n,
                     S.nslices, S.kbase, dspan);
  SGM_CHECK_LAUNCH();
  int32_t hspan = 0;
  SGM_HIP(hipMemcpyAsync(&hspan, dspan, sizeof(int32_t),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipStreamSynchronize(st));
  dfree(dspan);
  if (hspan <= 65535 && n >= 1) {
    S.rcol = dmalloc<int16_t>(total);
    hipLaunchKernelGGL(k_sell_rel16, dim3(grid1(S.nslices, wpb)),
                       dim3(wpb * kWave), 0, st, S.col, S.ptr, S.width,
                       S.kbase, n, S.nslices, S.rcol);
    SGM_CHECK_LAUNCH();
  } else {
    dfree(S.kbase);
  }
}

void sell_fill_values(const Sell& S, const double* val, hipStream_t st) {
  hipLaunchKernelGGL(k_sell_values, dim3(grid1(S.nnz_padded)), dim3(256), 0,
                     st, S.src, S.nnz_padded, val, S.val64, S.val32);
  SGM_CHECK_LAUNCH();
}

void sell_free(Sell& S) {
  dfree(S.ptr);
  dfree(S.width);
  dfree(S.col);
  dfree(S.rcol);
  dfree(S.kbase);
  dfree(S.src);
  dfree(S.val64);
  dfree(S.val32);
}

void matrix_extract_diag(Matrix& M, hipStream_t st) {
  hipLaunchKernelGGL(k_diag, dim3(grid1(M.n)), dim3(256), 0, st, M.row_ptr,
                     M.col, M.val, M.n, M.diag);
  SGM_CHECK_LAUNCH();
}

// max |column - row| over the nonzeros (integer maximum: deterministic)
__global__ void k_bandwidth(const int32_t* row_of, const int32_t* col,
                            int64_t nnz, int* out) {
  int m = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int d = col[k] - row_of[k];
    m = max(m, d < 0 ? -d : d);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
  if (threadIdx.x % kWave == 0) atomicMax(out, m);
}

Matrix* matrix_create(int64_t n, int64_t nnz, const int32_t* rp,
                      const int32_t* col, const double* val, hipStream_t st) {
  Matrix* M = new Matrix();
  M->n = n;
  M->nnz = nnz;
  int32_t* rpT = nullptr;
  int32_t* colT = nullptr;
  int32_t* permT = nullptr;
  int32_t* keys_out = nullptr;
  int32_t* iota = nullptr;
  int32_t* cnt = nullptr;
  char* tmp = nullptr;
  int* bad = nullptr;
  try {
    M->row_ptr = dmalloc<int32_t>(n + 1);
    M->col = dmalloc<int32_t>(nnz);
    M->row_of = dmalloc<int32_t>(nnz);
    M->val = dmalloc<double>(nnz);
    M->diag = dmalloc<double>(n);
    bad = dmalloc<int>(1);
    SGM_HIP(hipMemcpyAsync(M->row_ptr, rp, sizeof(int32_t) * (n + 1),
                           hipMemcpyDeviceToDevice, st));
    if (nnz > 0) {
      SGM_HIP(hipMemcpyAsync(M->col, col, sizeof(int32_t) * nnz,
                             hipMemcpyDeviceToDevice, st));
      SGM_HIP(hipMemcpyAsync(M->val, val, sizeof(double) * nnz,
                             hipMemcpyDeviceToDevice, st));
    }
    SGM_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_validate, dim3(grid1(n + 1)), dim3(256), 0, st,
                       M->row_ptr, M->col, n, nnz, bad);
    SGM_CHECK_LAUNCH();
    int hbad = 0;
    SGM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost,
                           st));
    SGM_HIP(hipStreamSynchronize(st));
    if (hbad)
      throw Error{SGM_EINVAL, "invalid CSR arrays (code " +
                                  std::to_string(hbad) + ")"};
    hipLaunchKernelGGL(k_row_of, dim3(grid1(n)), dim3(256), 0, st,
                       M->row_ptr, n, M->row_of);
    SGM_CHECK_LAUNCH();
    SGM_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    if (nnz > 0) {
      const int64_t gb = grid1(nnz) < 4096 ? grid1(nnz) : 4096;
      hipLaunchKernelGGL(k_bandwidth, dim3((unsigned)gb), dim3(256), 0, st,
                         M->row_of, M->col, nnz, bad);
      SGM_CHECK_LAUNCH();
    }
    int hbw = 0;
    SGM_HIP(hipMemcpyAsync(&hbw, bad, sizeof(int), hipMemcpyDeviceToHost,
                           st));
    SGM_HIP(hipStreamSynchronize(st));
    M->bandwidth = hbw;
    matrix_extract_diag(*M, st);
    // forward SELL
    sell_build(M->fwd, n, M->row_ptr, M->col, nullptr, st);
    sell_fill_values(M->fwd, M->val, st);
    // transpose: stable radix sort of (col, k) keeps row order in a column
    rpT = dmalloc<int32_t>(n + 1);
    colT = dmalloc<int32_t>(nnz);
    permT = dmalloc<int32_t>(nnz);
    keys_out = dmalloc<int32_t>(nnz);
    iota = dmalloc<int32_t>(nnz);
    cnt = dmalloc<int32_t>(n + 1);
    hipLaunchKernelGGL(k_iota, dim3(grid1(nnz)), dim3(256), 0, st, iota, nnz);
    SGM_CHECK_LAUNCH();
    int end_bit = 1;
    while (end_bit < 31 && ((int64_t)1 << end_bit) <= n) ++end_bit;
    size_t tb = 0;
    SGM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, M->col, keys_out,
                                               iota, permT, (int)nnz, 0,
                                               end_bit, st));
    tmp = dmalloc<char>((int64_t)tb);
    SGM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, M->col, keys_out,
                                               iota, permT, (int)nnz, 0,
                                               end_bit, st));
    SGM_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), st));
    hipLaunchKernelGGL(k_count, dim3(grid1(nnz)), dim3(256), 0, st, M->col,
                       nnz, cnt);
    SGM_CHECK_LAUNCH();
    size_t tb2 = 0;
    SGM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, cnt, rpT,
                                             (int)(n + 1), st));
    char* tmp2 = dmalloc<char>((int64_t)tb2);
    SGM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp2, tb2, cnt, rpT,
                                             (int)(n + 1), st));
    hipLaunchKernelGGL(k_gather_i32, dim3(grid1(nnz)), dim3(256), 0, st,
                       M->row_of, permT, nnz, colT);
    SGM_CHECK_LAUNCH();
    sell_build(M->trn, n, rpT, colT, permT, st);
    sell_fill_values(M->trn, M->val, st);
    SGM_HIP(hipStreamSynchronize(st));
    dfree(tmp2);
  } catch (...) {
    (void)hipStreamSynchronize(st);
    dfree(rpT); dfree(colT); dfree(permT); dfree(keys_out); dfree(iota);
    dfree(cnt); dfree(tmp); dfree(bad);
    sell_free(M->fwd);
    sell_free(M->trn);
    dfree(M->row_ptr); dfree(M->col); dfree(M->row_of); dfree(M->val);
    dfree(M->diag);
    delete M;
    throw;
  }
  dfree(rpT); dfree(colT); dfree(permT); dfree(keys_out); dfree(iota);
  dfree(cnt); dfree(tmp); dfree(bad);
  return M;
}

void matrix_update_values(Matrix* M, const double* val, hipStream_t st) {
  if (M->nnz > 0)
    SGM_HIP(hipMemcpyAsync(M->val, val, sizeof(double) * M->nnz,
                           hipMemcpyDeviceToDevice, st));
  matrix_extract_diag(*M, st);
  sell_fill_values(M->fwd, M->val, st);
  sell_fill_values(M->trn, M->val, st);
  // ILU(0) factors, when built, follow the values
  if (M->ilu) ilu_factor(*M, st);
}

void matrix_destroy(Matrix* M) {
  if (!M) return;
  (void)hipDeviceSynchronize();
  sell_free(M->fwd);
  sell_free(M->trn);
  ilu_free(M->ilu);
  dfree(M->row_ptr); dfree(M->col); dfree(M->row_of); dfree(M->val);
  dfree(M->diag);
  delete M;
}

}  // namespace sgm
