// Sparse mat-vec on SELL-C-64 (one wavefront per 64-row slice, fully
// coalesced value/index streams) with the epilogues the s-step cycle needs,
// plus the small vector kernels around it.
#include "internal.h"

namespace sgm {

namespace {

constexpr int kSpmvBlock = 256;                    // 4 wavefronts
constexpr int kSlicesPerBlock = kSpmvBlock / kWave;

// NQ consecutive entries k .. k + NQ - 1 of lane's row in one pass: all
// index and value loads go out together, then all NQ x gathers, then the
// products are added in entry order.
template <int NQ, typename T, typename IDX>
__device__ __forceinline__ void sell_pass(T& sum, int64_t base, int k,
                                          const IDX* __restrict__ col,
                                          const int32_t* __restrict__ kb,
                                          const T* __restrict__ val,
                                          QView<T> XV,
                                          const T* __restrict__ x, int lane) {
  int32_t c[NQ];
  T v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int64_t e = base + (int64_t)(k + q) * kSlice;
    if constexpr (sizeof(IDX) == 2)
      c[q] = kb[k + q] + lane + (int32_t)col[e];
    else
      c[q] = col[e];
    v[q] = val[e];
  }
  T xv[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) xv[q] = x[XV.row_off(c[q])];
#pragma unroll
  for (int q = 0; q < NQ; ++q) sum += v[q] * xv[q];
}

// Row r = 64 s + lane of A times x on SELL-C-64 slice s (0 for s past the
// last slice): the matrix part of every SpMV kernel below, so the fused
// matrix powers kernel computes bitwise the rows of the one-step kernel.
// IDX is int32_t (absolute columns) or int16_t (16-bit relative columns:
// group base kbase[ptr[s] / 64 + w] + lane + offset).  x is read at
// XV.row_off(column).  Passes of eight entries, then one pass of exactly
// the remaining 1..7 (a wavefront-uniform switch on the slice width, so
// stencil rows of 5 or 7 entries issue no padded loads).
template <typename T, typename IDX>
__device__ __forceinline__ T sell_row_dot(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ width,
    const IDX* __restrict__ col, const int32_t* __restrict__ kbase,
    const T* __restrict__ val, QView<T> XV, const T* __restrict__ x,
    int64_t nslices, int64_t s, int lane) {
  T sum = 0;
  if (s < nslices) {
    const int64_t p0 = ptr[s];
    const int64_t base = p0 + lane;
    const int w = width[s];
    const int32_t* __restrict__ kb =
        sizeof(IDX) == 2 ? kbase + (p0 >> 6) : nullptr;
    int k = 0;
    for (; k + 8 <= w; k += 8)
      sell_pass<8, T, IDX>(sum, base, k, col, kb, val, XV, x, lane);
    switch (w - k) {
      case 1: sell_pass<1, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      case 2: sell_pass<2, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      case 3: sell_pass<3, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      case 4: sell_pass<4, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      case 5: sell_pass<5, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      case 6: sell_pass<6, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      case 7: sell_pass<7, T, IDX>(sum, base, k, col, kb, val, XV, x, lane); break;
      default: break;
    }
  }
  return sum;
}

// The matrix powers recurrence of Eq. (newtonrecurrence) on row r:
// y = (sum - theta xo - delta xp) / gamma with (theta, gamma, delta) =
// rec[3 j .. 3 j + 2]; the delta term only when the previous vector is
// given.
template <typename T>
__device__ __forceinline__ T mpk_row(T sum, T xo, T xp, bool has_prev,
                                     const double* __restrict__ rec, int j) {
  const T theta = (T)rec[3 * j], gamma = (T)rec[3 * j + 1],
          delta = (T)rec[3 * j + 2];
  T v = sum - theta * xo;
  if (has_prev) v = v - delta * xp;
  return v / gamma;
}

// Fixed-order sum of q over the workgroup's lanes (wavefront tree, then the
// wavefronts in order), written to part[blockIdx.x].
__device__ __forceinline__ void block_partial(double q, double* part) {
  __shared__ double red[kSlicesPerBlock];
  for (int off = kWave / 2; off > 0; off >>= 1) q += __shfl_xor(q, off);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kSlicesPerBlock; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// x, xprev and y are columns of a block of vectors with layout XV (row r of
// a column at column base + XV.row_off(r)); the plain and residual
// epilogues use contiguous vectors (column-major view).  The matrix
// multiplies x itself, or (PREC) xm with layout XM: with a right
// preconditioner z = M^{-1} x while the recurrence's shift terms still use
// x.  GATED: the launch does nothing unless *gate == expect.  Both are
// separate instantiations: the few extra argument loads and waits at the
// start of every wavefront cost the other launches 3-5% on a 7-point
// stencil, whose wavefronts are short.  NORM (EPI_MPK): the workgroup's
// partial sum of y^2 (of the stored values, in float64) goes to
// part[blockIdx.x], the fused square-sum epilogue of the basis vectors.
template <typename T, int EPI, typename IDX, bool GATED = false,
          bool PREC = false, bool NORM = false>
__global__ __launch_bounds__(kSpmvBlock) void k_spmv(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ width,
    const IDX* __restrict__ col, const int32_t* __restrict__ kbase,
    const T* __restrict__ val, QView<T> XV, const T* __restrict__ x,
    QView<T> XM, const T* __restrict__ xm, const T* __restrict__ xprev,
    T* __restrict__ y, const double* __restrict__ b,
    double* __restrict__ part, int64_t n, int64_t nslices,
    const double* __restrict__ rec, int j, int xcd_contig,
    const int* __restrict__ gate, int expect) {
  // a step queued ahead of the result it depends on: nothing to do unless
  // the assumed block size was right
  if constexpr (GATED) {
    if (*gate != expect) return;
  }
  // Workgroup b runs on XCD b % 8.  With xcd_contig each XCD takes one
  // contiguous range of slices instead of every eighth group of four, so
  // the x lines that neighbouring slices share are fetched into one L2.
  // That pays when the matrix stays in the Infinity Cache; when it streams
  // from HBM the interleaved order measured faster.
  int64_t bl = blockIdx.x;
  if (xcd_contig) {
    const int64_t per = gridDim.x / 8;
    if (bl < per * 8) bl = (bl % 8) * per + bl / 8;
  }
  // slice index is wavefront-uniform: its metadata comes in scalar loads
  const int64_t s = bl * kSlicesPerBlock +
                    __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int64_t r = s * kSlice + lane;
  // the epilogue's own operands are loaded first, so their latency
  // overlaps the matrix stream instead of following it
  T xo = 0, xp = 0;
  int64_t ro = 0;
  double bb = 0.0;
  if constexpr (EPI == EPI_MPK) {
    if (r < n) {
      ro = XV.row_off(r);
      xo = x[ro];
      if (xprev != nullptr) xp = xprev[ro];
    }
  } else if constexpr (EPI == EPI_RESID) {
    if (r < n) bb = b[r];
  }
  T sum;
  if constexpr (PREC)
    sum = sell_row_dot<T, IDX>(ptr, width, col, kbase, val, XM, xm, nslices,
                               s, lane);
  else
    sum = sell_row_dot<T, IDX>(ptr, width, col, kbase, val, XV, x, nslices,
                               s, lane);
  if constexpr (EPI == EPI_PLAIN) {
    if (r < n) y[r] = sum;
  } else if constexpr (EPI == EPI_MPK) {
    T yv = 0;
    if (r < n) {
      yv = mpk_row<T>(sum, xo, xp, xprev != nullptr, rec, j);
      y[ro] = yv;
    }
    if constexpr (NORM) block_partial((double)yv * (double)yv, part);
  } else {  // EPI_RESID (float64): r = b - A x, partial sums of r^2
    double rr = 0.0;
    if (r < n) {
      rr = bb - (double)sum;
      y[r] = (T)rr;
    }
    block_partial(rr * rr, part);
  }
}

// One launch of the depth-k matrix powers kernel: up to kMaxMpkTasks
// (step, row slab) pieces, each the recurrence of one step on the slices
// [s0, s0 + ns) of one slab.  Piece t owns workgroups [wg[t], wg[t + 1]);
// every wg[t] is a multiple of 8, so a slab's slices fall on the same XCD
// (workgroup id mod 8) in every launch that touches the slab.
template <typename T, typename IDX>
__global__ __launch_bounds__(kSpmvBlock) void k_mpk_tasks(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ width,
    const IDX* __restrict__ col, const int32_t* __restrict__ kbase,
    const T* __restrict__ val, QView<T> XV, int64_t n, int64_t nslices,
    const double* __restrict__ rec, MpkTasks tasks) {
  const int bid = (int)blockIdx.x;
  // the piece's fields, selected with constant indices (a run-time index
  // into the argument struct would copy it to scratch memory)
  int64_t s0 = tasks.t[0].s0, ns = tasks.t[0].ns;
  int wg0 = tasks.wg[0], xcol = tasks.t[0].xcol, pcol = tasks.t[0].pcol,
      ycol = tasks.t[0].ycol, jrec = tasks.t[0].j;
#pragma unroll
  for (int u = 1; u < kMaxMpkTasks; ++u)
    if (u < tasks.count && bid >= tasks.wg[u]) {
      s0 = tasks.t[u].s0;
      ns = tasks.t[u].ns;
      wg0 = tasks.wg[u];
      xcol = tasks.t[u].xcol;
      pcol = tasks.t[u].pcol;
      ycol = tasks.t[u].ycol;
      jrec = tasks.t[u].j;
    }
  const int64_t local = (int64_t)(bid - wg0) * kSlicesPerBlock +
                        __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (local >= ns) return;
  const int64_t s = s0 + local;
  const int lane = threadIdx.x % kWave;
  const int64_t r = s * kSlice + lane;
  const T* x = XV.col(xcol);
  const T* xprev = pcol >= 0 ? (const T*)XV.col(pcol) : nullptr;
  T xo = 0, xp = 0;
  int64_t ro = 0;
  if (r < n) {
    ro = XV.row_off(r);
    xo = x[ro];
    if (xprev != nullptr) xp = xprev[ro];
  }
  const T sum = sell_row_dot<T, IDX>(ptr, width, col, kbase, val, XV, x,
                                     nslices, s, lane);
  if (r < n)
    XV.col(ycol)[ro] = mpk_row<T>(sum, xo, xp, xprev != nullptr, rec, jrec);
}

inline unsigned spmv_grid(const Sell& S) {
  return (unsigned)ceil_div(S.nslices, kSlicesPerBlock);
}

// Matrices whose SELL values and indices fit in 192 MiB stay in the 256 MB
// Infinity Cache across back-to-back SpMVs: XCD-contiguous slice ranges
// (measured on the 7-point 128^3 stencil: 29.0 -> 26.6 us in float64).
// Larger ones stream from HBM, where the interleaved order measured 4-5%
// faster (192^3 and 4096^2 stencils).
inline int xcd_contig(const Sell& S, int vbytes) {
  const int64_t bytes = S.nnz_padded * (vbytes + (S.rcol ? 2 : 4));
  return bytes <= ((int64_t)192 << 20) ? 1 : 0;
}

// out[0] = the fixed-order sum of part[0:np].
__global__ __launch_bounds__(1024) void k_sum_partials(const double* part,
                                                       int64_t np,
                                                       double* out) {
  __shared__ double red[1024];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 1024) t += part[i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(1024) void k_reduce_norm(const double* part,
                                                      int64_t np,
                                                      double* out) {
  __shared__ double red[1024];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 1024) t += part[i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

template <typename T>
__global__ void k_scale_into(const double* r, const double* beta, QView<T> Q,
                             int c, int64_t n, int64_t ld) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ld) return;
  *Q.at(i, c) = i < n ? (T)(r[i] / beta[0]) : (T)0;
}

template <typename T>
__global__ void k_zero_pad(QView<T> Q, int64_t n, int64_t ld, int ncols) {
  int64_t pad = ld - n;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= pad * ncols) return;
  int64_t c = t / pad, r = n + t % pad;
  *Q.at(r, c) = (T)0;
}

__global__ void k_jacobi_values(const int64_t* src, const int32_t* col,
                                int64_t m, const double* val,
                                const double* diag, double* v64, float* v32) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  int64_t k = src[e];
  double v = k >= 0 ? val[k] / diag[col[e]] : 0.0;
  v64[e] = v;
  v32[e] = (float)v;
}

__global__ void k_vec_scale(double* x, const double* d, int64_t n,
                            int divide) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = divide ? x[i] / d[i] : x[i] * d[i];
}

__global__ void k_grad_vals(const int32_t* row_of, const int32_t* col,
                            int64_t nnz, const double* lam, const double* x,
                            double* g) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  g[k] = -lam[row_of[k]] * x[col[k]];
}

__global__ void k_cast(const double* a, float* b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_copy(const double* a, double* b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ void k_axpy(const double* z, double* x, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += z[i];
}

inline unsigned g1(int64_t n) {
  return (unsigned)ceil_div(n > 0 ? n : 1, 256);
}

}  // namespace

template <typename T>
void spmv_plain(const Sell& S, const T* val, const T* x, T* y,
                hipStream_t st) {
#define SGM_SPMV(IDX, colp)                                                   \
  hipLaunchKernelGGL((k_spmv<T, EPI_PLAIN, IDX>), dim3(spmv_grid(S)),         \
                     dim3(kSpmvBlock), 0, st, S.ptr, S.width, colp, S.kbase,  \
                     val, colmajor_view<T>(nullptr, 0), x,                    \
                     colmajor_view<T>(nullptr, 0), x, (const T*)nullptr,      \
                     y, (const double*)nullptr, (double*)nullptr, S.n,        \
                     S.nslices, (const double*)nullptr, 0,                    \
                     xcd_contig(S, (int)sizeof(T)), (const int*)nullptr, 0)
  if (S.rcol) SGM_SPMV(int16_t, S.rcol); else SGM_SPMV(int32_t, S.col);
#undef SGM_SPMV
  SGM_CHECK_LAUNCH();
}

template <typename T>
void spmv_mpk(const Sell& S, const T* val, QView<T> Q, int jx, int jprev,
              int jy, const double* rec, int j, hipStream_t st,
              const int* gate, int expect) {
  const T* xp = jprev >= 0 ? (const T*)Q.col(jprev) : (const T*)nullptr;
#define SGM_SPMV(IDX, G, colp)                                                \
  hipLaunchKernelGGL((k_spmv<T, EPI_MPK, IDX, G>), dim3(spmv_grid(S)),        \
                     dim3(kSpmvBlock), 0, st, S.ptr, S.width, colp, S.kbase,  \
                     val, Q, (const T*)Q.col(jx), Q, (const T*)Q.col(jx), xp, \
                     Q.col(jy), (const double*)nullptr, (double*)nullptr,     \
                     S.n, S.nslices, rec, j, xcd_contig(S, (int)sizeof(T)),  \
                     gate, expect)
  if (gate != nullptr) {
    if (S.rcol) SGM_SPMV(int16_t, true, S.rcol);
    else SGM_SPMV(int32_t, true, S.col);
  } else {
    if (S.rcol) SGM_SPMV(int16_t, false, S.rcol);
    else SGM_SPMV(int32_t, false, S.col);
  }
#undef SGM_SPMV
  SGM_CHECK_LAUNCH();
}

template <typename T>
void spmv_mpk_norm(const Sell& S, const T* val, QView<T> Q, int jx, int jprev,
                   int jy, const double* rec, int j, double* part,
                   double* norm2, hipStream_t st) {
  const T* xp = jprev >= 0 ? (const T*)Q.col(jprev) : (const T*)nullptr;
#define SGM_SPMV(IDX, colp)                                                   \
  hipLaunchKernelGGL((k_spmv<T, EPI_MPK, IDX, false, false, true>),           \
                     dim3(spmv_grid(S)), dim3(kSpmvBlock), 0, st, S.ptr,      \
                     S.width, colp, S.kbase, val, Q, (const T*)Q.col(jx), Q,  \
                     (const T*)Q.col(jx), xp, Q.col(jy),                      \
                     (const double*)nullptr, part, S.n, S.nslices, rec, j,    \
                     xcd_contig(S, (int)sizeof(T)), (const int*)nullptr, 0)
  if (S.rcol) SGM_SPMV(int16_t, S.rcol); else SGM_SPMV(int32_t, S.col);
#undef SGM_SPMV
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st,
                     (const double*)part, (int64_t)spmv_grid(S), norm2);
  SGM_CHECK_LAUNCH();
}

template void spmv_mpk_norm<double>(const Sell&, const double*, QView<double>,
                                    int, int, int, const double*, int,
                                    double*, double*, hipStream_t);
template void spmv_mpk_norm<float>(const Sell&, const float*, QView<float>,
                                   int, int, int, const double*, int, double*,
                                   double*, hipStream_t);

// Depth-k matrix powers kernel (temporal blocking).  The rows are cut into
// slabs of at least the matrix bandwidth h (|column - row| <= h), so step
// j on slab S reads step j - 1's vector only on slabs S - 1 .. S + 1.
// Launch L runs step j on slab L - 2 j for every step j of the group that
// has such a slab: each piece then depends only on pieces of earlier
// launches (step j - 1 on slabs up to S + 1 ran in launch S + 1 + 2 (j - 1)
// = L - 1), and a slab's matrix rows are read again two launches after
// their previous use, while still in the caches.  Rows are computed
// exactly as by the one-step kernel.
MpkPlan mpk_plan(const Sell& S, int64_t bandwidth, int depth, int vbytes) {
  MpkPlan p;
  p.depth = depth < 1 ? 1 : (depth > kMaxMpkTasks ? kMaxMpkTasks : depth);
  if (p.depth == 1 || S.nslices < 1) {
    p.depth = 1;
    return p;
  }
  // slab: at least the bandwidth, at least 1024 slices (a launch of four
  // pieces then has about 1000 workgroups), about 8 MB of matrix values and
  // indices (two launches' worth of slabs then stay in the 256 MB Infinity
  // Cache between a slab's uses)
  const int64_t per_slice =
      ceil_div(S.nnz_padded, S.nslices) * (vbytes + (S.rcol ? 2 : 4));
  int64_t ns = ceil_div(bandwidth + 1, kSlice);
  int64_t target = ((int64_t)8 << 20) / (per_slice > 0 ? per_slice : 1);
  if (target < 1024) target = 1024;
  if (ns < target) ns = target;
  ns = round_up(ns, kSlicesPerBlock);
  const int64_t G = ceil_div(S.nslices, ns);
  if (G < 3) {
    p.depth = 1;  // too few slabs to overlap
    return p;
  }
  p.slab_slices = ns;
  p.nslabs = G;
  return p;
}

template <typename T>
void spmv_mpk_steps(const Sell& S, const T* val, QView<T> Q,
                    const MpkStep* steps, int nsteps, const double* rec,
                    const MpkPlan& plan, hipStream_t st) {
  if (nsteps <= 0) return;
  if (plan.depth <= 1) {
    for (int j = 0; j < nsteps; ++j)
      spmv_mpk<T>(S, val, Q, steps[j].xcol, steps[j].pcol, steps[j].ycol, rec,
                  steps[j].j, st);
    return;
  }
  const int64_t G = plan.nslabs, ns = plan.slab_slices;
  for (int j0 = 0; j0 < nsteps; j0 += plan.depth) {
    const int k = nsteps - j0 < plan.depth ? nsteps - j0 : plan.depth;
    for (int64_t L = 0; L < G + 2 * (k - 1); ++L) {
      MpkTasks tasks;
      tasks.count = 0;
      int wg = 0;
      for (int jj = k - 1; jj >= 0; --jj) {  // oldest step first
        const int64_t slab = L - 2 * jj;
        if (slab < 0 || slab >= G) continue;
        MpkTask& t = tasks.t[tasks.count];
        t.s0 = slab * ns;
        t.ns = (slab + 1) * ns <= S.nslices ? ns : S.nslices - slab * ns;
        t.xcol = steps[j0 + jj].xcol;
        t.pcol = steps[j0 + jj].pcol;
        t.ycol = steps[j0 + jj].ycol;
        t.j = steps[j0 + jj].j;
        tasks.wg[tasks.count] = wg;
        wg += (int)round_up(ceil_div(t.ns, kSlicesPerBlock), 8);
        ++tasks.count;
      }
      for (int u = tasks.count; u <= kMaxMpkTasks; ++u) tasks.wg[u] = wg;
#define SGM_MPKT(IDX, colp)                                                   \
  hipLaunchKernelGGL((k_mpk_tasks<T, IDX>), dim3((unsigned)wg),               \
                     dim3(kSpmvBlock), 0, st, S.ptr, S.width, colp, S.kbase,  \
                     val, Q, S.n, S.nslices, rec, tasks)
      if (S.rcol) SGM_MPKT(int16_t, S.rcol); else SGM_MPKT(int32_t, S.col);
#undef SGM_MPKT
      SGM_CHECK_LAUNCH();
    }
  }
}

void spmv_mpk_prec(const Sell& S, const double* val, QView<double> Q,
                   const double* z, int jx, int jprev, int jy,
                   const double* rec, int j, hipStream_t st) {
  const double* xp =
      jprev >= 0 ? (const double*)Q.col(jprev) : (const double*)nullptr;
#define SGM_SPMV(IDX, colp)                                                   \
  hipLaunchKernelGGL((k_spmv<double, EPI_MPK, IDX, false, true>),             \
                     dim3(spmv_grid(S)),                                      \
                     dim3(kSpmvBlock), 0, st, S.ptr, S.width, colp, S.kbase,  \
                     val, Q, (const double*)Q.col(jx),                        \
                     colmajor_view<double>(nullptr, 0), z, xp, Q.col(jy),     \
                     (const double*)nullptr, (double*)nullptr, S.n,           \
                     S.nslices, rec, j, xcd_contig(S, (int)sizeof(double)),  \
                     (const int*)nullptr, 0)
  if (S.rcol) SGM_SPMV(int16_t, S.rcol); else SGM_SPMV(int32_t, S.col);
#undef SGM_SPMV
  SGM_CHECK_LAUNCH();
}

template void spmv_mpk_steps<double>(const Sell&, const double*,
                                     QView<double>, const MpkStep*, int,
                                     const double*, const MpkPlan&,
                                     hipStream_t);
template void spmv_mpk_steps<float>(const Sell&, const float*, QView<float>,
                                    const MpkStep*, int, const double*,
                                    const MpkPlan&, hipStream_t);

int64_t resid_partials(const Sell& S) { return spmv_grid(S); }

int64_t spmv_resid(const Sell& S, const double* val, const double* x,
                   const double* b, double* r, double* part, hipStream_t st) {
#define SGM_SPMV(IDX, colp)                                                   \
  hipLaunchKernelGGL((k_spmv<double, EPI_RESID, IDX>), dim3(spmv_grid(S)),    \
                     dim3(kSpmvBlock), 0, st, S.ptr, S.width, colp, S.kbase,  \
                     val, colmajor_view<double>(nullptr, 0), x,               \
                     colmajor_view<double>(nullptr, 0), x,                    \
                     (const double*)nullptr, r, b, part, S.n, S.nslices,      \
                     (const double*)nullptr, 0, 0, (const int*)nullptr, 0)
  if (S.rcol) SGM_SPMV(int16_t, S.rcol); else SGM_SPMV(int32_t, S.col);
#undef SGM_SPMV
  SGM_CHECK_LAUNCH();
  return spmv_grid(S);
}

template void spmv_plain<double>(const Sell&, const double*, const double*,
                                 double*, hipStream_t);
template void spmv_plain<float>(const Sell&, const float*, const float*,
                                float*, hipStream_t);
template void spmv_mpk<double>(const Sell&, const double*, QView<double>, int,
                               int, int, const double*, int, hipStream_t,
                               const int*, int);
template void spmv_mpk<float>(const Sell&, const float*, QView<float>, int,
                              int, int, const double*, int, hipStream_t,
                              const int*, int);

void reduce_norm(const double* part, int64_t np, double* out,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_norm, dim3(1), dim3(1024), 0, st, part, np,
                     out);
  SGM_CHECK_LAUNCH();
}

template <typename T>
void scale_into(const double* r, const double* beta, QView<T> Q, int c,
                int64_t n, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_into<T>, dim3(g1(ld)), dim3(256), 0, st, r,
                     beta, Q, c, n, ld);
  SGM_CHECK_LAUNCH();
}
template void scale_into<double>(const double*, const double*, QView<double>,
                                 int, int64_t, int64_t, hipStream_t);
template void scale_into<float>(const double*, const double*, QView<float>,
                                int, int64_t, int64_t, hipStream_t);

template <typename T>
void zero_pad_rows(QView<T> Q, int64_t n, int64_t ld, int ncols,
                   hipStream_t st) {
  if (ld <= n || ncols <= 0) return;
  hipLaunchKernelGGL(k_zero_pad<T>, dim3(g1((ld - n) * ncols)), dim3(256), 0,
                     st, Q, n, ld, ncols);
  SGM_CHECK_LAUNCH();
}
template void zero_pad_rows<double>(QView<double>, int64_t, int64_t, int,
                                    hipStream_t);
template void zero_pad_rows<float>(QView<float>, int64_t, int64_t, int,
                                   hipStream_t);

void jacobi_values(const Matrix& M, const Sell& S, double* v64, float* v32,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_values, dim3(g1(S.nnz_padded)), dim3(256), 0,
                     st, S.src, S.col, S.nnz_padded, M.val, M.diag, v64, v32);
  SGM_CHECK_LAUNCH();
}

void vec_scale_div(double* x, const double* d, int64_t n, bool divide,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_vec_scale, dim3(g1(n)), dim3(256), 0, st, x, d, n,
                     divide ? 1 : 0);
  SGM_CHECK_LAUNCH();
}

void grad_vals(const Matrix& M, const double* lam, const double* x,
               double* g, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_vals, dim3(g1(M.nnz)), dim3(256), 0, st,
                     M.row_of, M.col, M.nnz, lam, x, g);
  SGM_CHECK_LAUNCH();
}

void cast_f64_f32(const double* a, float* b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast, dim3(g1(n)), dim3(256), 0, st, a, b, n);
  SGM_CHECK_LAUNCH();
}

void axpy_f64(const double* z, double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(g1(n)), dim3(256), 0, st, z, x, n);
  SGM_CHECK_LAUNCH();
}

void copy_f64(const double* a, double* b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(g1(n)), dim3(256), 0, st, a, b, n);
  SGM_CHECK_LAUNCH();
}

}  // namespace sgm
