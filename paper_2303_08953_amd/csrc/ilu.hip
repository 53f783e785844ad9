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
// bandwidth.
//
// Within a level the rows are sorted, and each row's strict triangle is
// stored per position in level order (ELL: entry t of position p at
// t * n + p), so a level's threads read consecutive addresses.  Each entry
// also records the position of the row it refers to, and the solve keeps
// the values of the last kRing positions in an LDS ring: dependencies on
// recent levels (all of them for stencils whose levels are small) are read
// from LDS, older ones from global memory.  The next level's structure and
// right-hand side are loaded before the barrier that ends the current one,
// so a level costs LDS reads, its arithmetic and the barrier.
#include "internal.h"

#include <algorithm>
#include <vector>

#include <hipcub/hipcub.hpp>

namespace sgm {

namespace {

constexpr int kIluBlock = 1024;  // factorisation; solves use 512 or 1024
constexpr int kLevDeps = 8;   // dependencies a row keeps in registers
constexpr int kRing = 16384;  // solved values kept in LDS (128 KiB)

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

__global__ void k_inverse_perm(const int32_t* rows, int64_t n,
                               int32_t* pos) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) pos[rows[p]] = (int32_t)p;
}

// The strict triangle of each position's row in level order (ELL): column,
// CSR index and the column's own position in level order.
__global__ void k_ilu_ell(const int32_t* rp, const int32_t* col,
                          const int32_t* dpos, const int32_t* rows,
                          const int32_t* pos, int64_t n, int upper,
                          int32_t wpad, int32_t* cnt, int32_t* ecol,
                          int32_t* epos, int32_t* esrc) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t i = rows[p];
  int32_t e0, e1;
  tri_range(rp, dpos, i, upper, e0, e1);
  cnt[p] = e1 - e0;
  for (int32_t t = 0; t < wpad; ++t) {
    const bool in = t < e1 - e0;
    const int64_t q = (int64_t)t * n + p;
    ecol[q] = in ? col[e0 + t] : 0;
    epos[q] = in ? pos[col[e0 + t]] : 0;
    esrc[q] = in ? e0 + t : -1;
  }
}

// far[0] = 1 when some entry depends on a position that the LDS ring no
// longer holds while its level is solved (position < end of the level -
// kRing); the solve then reads it from global memory and needs the full
// barrier between levels.
__global__ void k_ilu_far(const int32_t* key, const int32_t* lptr,
                          const int32_t* cnt, const int32_t* epos, int64_t n,
                          int32_t* far) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t lo = (int64_t)lptr[key[p] + 1] - kRing;
  bool f = false;
  for (int t = 0; t < cnt[p]; ++t)
    if (epos[(int64_t)t * n + p] < lo) f = true;
  if (f) far[0] = 1;
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
  const int32_t* lptr;  // [nlev + 1] level starts
  const int32_t* cnt;   // entries per position
  const int32_t* epos;  // [wpad * n] positions of the dependencies
  const double* eval;   // [wpad * n] factor values (0 in the padding)
  const int32_t* dest;  // forward: the row's backward position; backward:
                        // the row itself
};

// What one thread needs for one position of a level: every load depends on
// the position only (right-hand sides are kept in level order), so the loads
// of later levels go out before the current level is solved.  W entries of
// the row are loaded ahead (W >= the widest row for the common widths).
template <int W>
struct IluRow {
  int c, dest;
  double rhs, dv;
  int dp[W];
  double v[W];
};

// Loads for position p of the level that ends at p1; a thread with no
// position there loads the level's last one instead (always valid, nothing
// is stored for it), so every thread issues the same loads.
template <bool UPPER, int W>
__device__ __forceinline__ void ilu_load(const IluSide& S,
                                         const double* __restrict__ rhs,
                                         const double* __restrict__ dinv,
                                         int p, int p1, int64_t n,
                                         IluRow<W>& w) {
  const int pc = p < p1 ? p : p1 - 1;
  w.c = S.cnt[pc];
  w.dest = S.dest[pc];
  w.rhs = rhs[pc];
  w.dv = UPPER ? dinv[pc] : 1.0;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const int64_t q = (int64_t)t * n + pc;
    w.dp[t] = S.epos[q];
    w.v[t] = S.eval[q];
  }
}

// The value at dependency position dp: from the LDS ring, or with FAR from
// the phase's level-ordered values in global memory (gval) when the ring
// no longer holds it.  Both loads are issued and the value is selected, so
// no pointer mixes the LDS and global address spaces.
template <bool FAR>
__device__ __forceinline__ double ilu_dep(const double* ring,
                                          const double* gval, int dp,
                                          int lo) {
  const double yr = ring[dp & (kRing - 1)];
  if constexpr (FAR) {
    const double yg = gval[dp];
    return dp >= lo ? yr : yg;
  } else {
    return yr;
  }
}

// (rhs - sum_t v_t y(dep_t)) * dv for one position; entries past W (rows
// wider than the loads ahead) are read here.
template <bool FAR, int W>
__device__ __forceinline__ double ilu_solve_row(const IluSide& S,
                                                const IluRow<W>& w, int p,
                                                const double* ring,
                                                const double* gval, int lo,
                                                int64_t n) {
  double s = w.rhs;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    const double y = ilu_dep<FAR>(ring, gval, w.dp[t], lo);
    s -= w.v[t] * (t < w.c ? y : 0.0);
  }
  for (int t = W; t < w.c; ++t) {
    const int64_t q = (int64_t)t * n + p;
    s -= S.eval[q] * ilu_dep<FAR>(ring, gval, S.epos[q], lo);
  }
  return s * w.dv;
}

// Barrier that orders LDS only: the values a level hands to the next go
// through the ring, so its global stores (and the later levels' loads
// issued ahead) stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Levels whose loads are in flight: as many as the registers allow without
// spilling (four sets of two-entry rows, two of four-entry rows; rows of
// eight load at their own level).
template <int W>
constexpr int ahead() {
  return W <= 2 ? 3 : (W <= 4 ? 1 : 0);
}

// One substitution over its levels.  rhs: right-hand sides in this side's
// level order; lp: its level starts (in LDS); the value of position p goes
// to ring slot p mod kRing and to out[dest(p)] (the backward side's
// right-hand side, or the result z); with FAR also to gval[p].  During
// level [p0, p1) the slots written are those of p0 .. p1 - 1, which held
// positions below p1 - kRing, so every dependency at position >= lo =
// p1 - kRing is intact in the ring.  Without far dependencies the levels
// are separated by the LDS-only barrier; with them by the full one, which
// makes gval of earlier levels visible.  The loads of level l + ahead<W>()
// go out while level l is solved, into one of ahead<W>() + 1 register sets
// used in rotation (no register is copied while its load is in flight).
template <bool UPPER, bool FAR, int W, int BS>
__device__ __forceinline__ void ilu_phase(const IluSide& S, const int* lp,
                                          int nl, const double* rhs,
                                          const double* dinv, double* gval,
                                          double* out, double* ring,
                                          int64_t n) {
  constexpr int kAhead = ahead<W>();
  const int tid = (int)threadIdx.x;
  // level bounds, clamped past the last level (an empty range there loads
  // the last position and stores nothing)
  auto lstart = [&](int l) { return lp[l < nl ? l : nl]; };
  auto lend = [&](int l) { return lp[l < nl ? l + 1 : nl]; };
  IluRow<W> set[kAhead + 1];
#pragma unroll
  for (int k = 0; k < kAhead; ++k)
    ilu_load<UPPER, W>(S, rhs, dinv, lstart(k) + tid, lend(k), n, set[k]);
  for (int l0 = 0; l0 < nl; l0 += kAhead + 1) {
#pragma unroll
    for (int k = 0; k <= kAhead; ++k) {
      const int l = l0 + k;
      if (l < nl) {
        ilu_load<UPPER, W>(S, rhs, dinv, lstart(l + kAhead) + tid,
                           lend(l + kAhead), n, set[(k + kAhead) % (kAhead + 1)]);
        const int p0 = lp[l], p1 = lp[l + 1];
        const int lo = p1 - kRing;
        const int p = p0 + tid;
        const IluRow<W>& cur = set[k];
        const double v = ilu_solve_row<FAR, W>(S, cur, p, ring, gval, lo, n);
        if (p < p1) {
          ring[p & (kRing - 1)] = v;
          out[cur.dest] = v;
          if (FAR) gval[p] = v;
        }
        for (int pp = p + BS; pp < p1; pp += BS) {
          IluRow<W> w;
          ilu_load<UPPER, W>(S, rhs, dinv, pp, p1, n, w);
          const double v2 =
              ilu_solve_row<FAR, W>(S, w, pp, ring, gval, lo, n);
          ring[pp & (kRing - 1)] = v2;
          out[w.dest] = v2;
          if (FAR) gval[pp] = v2;
        }
        if (FAR)
          __syncthreads();
        else
          lds_barrier();
      }
    }
  }
}

template <int W, int BS>
__device__ __forceinline__ void ilu_apply_w(
    QView<const double> BV, const double* b, double* z, const IluSide& L,
    const IluSide& U, const int32_t* rows_l, const double* dinv,
    const int32_t* nlev, double* tl, double* tu, int64_t n, double* ring,
    int* lpl, int* lpu) {
  const int nl = nlev[0], nu = nlev[1];
  if (nlev[2])
    ilu_phase<false, true, W, BS>(L, lpl, nl, tl, dinv, tl, tu, ring, n);
  else
    ilu_phase<false, false, W, BS>(L, lpl, nl, tl, dinv, tl, tu, ring, n);
  // the backward substitution reads the forward one's values from tu
  __syncthreads();
  if (nlev[3])
    ilu_phase<true, true, W, BS>(U, lpu, nu, tu, dinv, tu, z, ring, n);
  else
    ilu_phase<true, false, W, BS>(U, lpu, nu, tu, dinv, tu, z, ring, n);
}

// z = M^{-1} b: b (read at BV.row_off(row); it may be z itself) has been
// gathered into the forward substitution's level order (tl); the forward
// substitution L y = b leaves y in the backward side's level order (tu),
// the backward substitution U z = y writes z by row.  tl and tu also hold
// each side's values by position for dependencies the ring has dropped.
// Both sides' level starts are copied into LDS (they fit for up to
// kLevLds - 2 levels in all; more levels take the global-memory variant).
// W: entries per row loaded ahead (2, 4 or 8, at least the wider side's
// widest row when that is at most 8).
constexpr int kLevLds = 7936;  // level starts kept in LDS (31 KiB)

template <int W, bool LPLDS, int BS>
__global__ __launch_bounds__(BS) void k_ilu_apply(
    QView<const double> BV, const double* b, double* z, IluSide L, IluSide U,
    const int32_t* __restrict__ rows_l, const double* __restrict__ dinv,
    const int32_t* __restrict__ nlev, double* tl, double* tu, int64_t n) {
  __shared__ double ring[kRing];
  __shared__ int lps[LPLDS ? kLevLds : 1];
  const int tid = (int)threadIdx.x;
  for (int i = tid; i < kRing; i += BS) ring[i] = 0.0;
  const int nl = nlev[0], nu = nlev[1];
  int* lpl = const_cast<int*>(L.lptr);
  int* lpu = const_cast<int*>(U.lptr);
  if constexpr (LPLDS) {
    for (int i = tid; i <= nl; i += BS) lps[i] = L.lptr[i];
    for (int i = tid; i <= nu; i += BS) lps[nl + 1 + i] = U.lptr[i];
    lpl = lps;
    lpu = lps + nl + 1;
  }
  __syncthreads();
  ilu_apply_w<W, BS>(BV, b, z, L, U, rows_l, dinv, nlev, tl, tu, n, ring,
                     lpl, lpu);
}

// tl[p] = b at the row of forward position p (the whole chip, before the
// single-workgroup solve).
__global__ void k_ilu_gather(QView<const double> BV, const double* b,
                             const int32_t* rows_l, double* tl, int64_t n) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) tl[p] = b[BV.row_off(rows_l[p])];
}

__global__ void k_compose(const int32_t* rows_l, const int32_t* pos_u,
                          int64_t n, int32_t* l2u) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) l2u[p] = pos_u[rows_l[p]];
}

// Entries per row that the solve loads ahead: 2, 4 or 8, the smallest
// that covers the widest row (8 beyond that; wider rows read the rest
// directly).
inline int apply_width(int width) {
  return width <= 2 ? 2 : (width <= 4 ? 4 : 8);
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
                IluLevels& S, int32_t* nlev_dev, int32_t* far_dev,
                hipStream_t st) {
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
  std::vector<int32_t> hl(S.nlev + 1);
  SGM_HIP(hipMemcpyAsync(hl.data(), S.lptr, sizeof(int32_t) * hl.size(),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipStreamSynchronize(st));
  S.max_level = 0;
  for (int32_t l = 0; l < S.nlev; ++l)
    S.max_level = std::max(S.max_level, hl[l + 1] - hl[l]);
  // at least as many columns as the solve loads ahead per row (2, 4 or 8)
  S.wpad = S.width > apply_width(S.width) ? S.width : apply_width(S.width);
  const int64_t wn = (int64_t)S.wpad * n;
  S.cnt = dalloc<int32_t>(n);
  S.ecol = dalloc<int32_t>(wn);
  S.epos = dalloc<int32_t>(wn);
  S.esrc = dalloc<int32_t>(wn);
  S.eval = dalloc<double>(wn);
  int32_t* pos = iota;  // the unsorted row numbers are no longer needed
  hipLaunchKernelGGL(k_inverse_perm, dim3(g256(n)), dim3(256), 0, st,
                     S.rows, n, pos);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ilu_ell, dim3(g256(n)), dim3(256), 0, st, M.row_ptr,
                     M.col, dpos, S.rows, pos, n, upper, S.wpad, S.cnt,
                     S.ecol, S.epos, S.esrc);
  SGM_CHECK_LAUNCH();
  SGM_HIP(hipMemsetAsync(far_dev, 0, sizeof(int32_t), st));
  hipLaunchKernelGGL(k_ilu_far, dim3(g256(n)), dim3(256), 0, st, key, S.lptr,
                     S.cnt, S.epos, n, far_dev);
  SGM_CHECK_LAUNCH();
  SGM_HIP(hipStreamSynchronize(st));
  for (void* p : {(void*)lev, (void*)key, (void*)iota, (void*)wdev, tmp})
    (void)hipFree(p);
}

void free_side(IluLevels& S) {
  for (void* p : {(void*)S.rows, (void*)S.lptr, (void*)S.cnt,
                  (void*)S.ecol, (void*)S.epos, (void*)S.esrc,
                  (void*)S.eval})
    if (p) (void)hipFree(p);
  S = IluLevels{};
}

}  // namespace

void ilu_free(Ilu*& I) {
  if (!I) return;
  free_side(I->L);
  free_side(I->U);
  for (void* p : {(void*)I->dpos, (void*)I->fac, (void*)I->dinv,
                  (void*)I->nlev_dev, (void*)I->flags, (void*)I->l2u,
                  (void*)I->tl, (void*)I->tu})
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
                     I.L.esrc, I.L.cnt, n, I.L.wpad, I.fac, I.L.eval);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_ilu_ell_vals, dim3(g256(n)), dim3(256), 0, st,
                     I.U.esrc, I.U.cnt, n, I.U.wpad, I.fac, I.U.eval);
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
    I.nlev_dev = dalloc<int32_t>(4);
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
    build_side(M, I.dpos, 0, I.L, I.nlev_dev, I.nlev_dev + 2, st);
    build_side(M, I.dpos, 1, I.U, I.nlev_dev + 1, I.nlev_dev + 3, st);
    I.max_level = std::max(I.L.max_level, I.U.max_level);
    I.l2u = dalloc<int32_t>(n);
    I.tl = dalloc<double>(n);
    I.tu = dalloc<double>(n);
    int32_t* pos_u = dalloc<int32_t>(n);
    hipLaunchKernelGGL(k_inverse_perm, dim3(g256(n)), dim3(256), 0, st,
                       I.U.rows, n, pos_u);
    SGM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_compose, dim3(g256(n)), dim3(256), 0, st, I.L.rows,
                       pos_u, n, I.l2u);
    SGM_CHECK_LAUNCH();
    SGM_HIP(hipStreamSynchronize(st));
    (void)hipFree(pos_u);
    ilu_factor(M, st);
  } catch (...) {
    ilu_free(M.ilu);
    throw;
  }
}

void ilu_apply(const Ilu& I, int64_t n, QView<const double> BV,
               const double* b, double* z, hipStream_t st) {
  const IluSide L{I.L.lptr, I.L.cnt, I.L.epos, I.L.eval, I.l2u};
  const IluSide U{I.U.lptr, I.U.cnt, I.U.epos, I.U.eval, I.U.rows};
  hipLaunchKernelGGL(k_ilu_gather, dim3(g256(n)), dim3(256), 0, st, BV, b,
                     (const int32_t*)I.L.rows, I.tl, n);
  SGM_CHECK_LAUNCH();
  const int w = apply_width(I.L.width > I.U.width ? I.L.width : I.U.width);
  const bool lds = (int64_t)I.L.nlev + I.U.nlev + 2 <= kLevLds;
  // 512 threads when every level fits (fewer waves meet at each barrier:
  // 474 against 738 ns per level on the 400^2 5-point grid), else 1024
  const bool small = I.max_level <= 512;
#define SGM_ILU(W, LDS, BS)                                                   \
  hipLaunchKernelGGL((k_ilu_apply<W, LDS, BS>), dim3(1), dim3(BS), 0, st, BV, \
                     b, z, L, U, (const int32_t*)I.L.rows,                    \
                     (const double*)I.dinv, (const int32_t*)I.nlev_dev, I.tl, \
                     I.tu, n)
#define SGM_ILU_BS(W, LDS)                                                    \
  do {                                                                        \
    if (small) SGM_ILU(W, LDS, 512); else SGM_ILU(W, LDS, 1024);              \
  } while (0)
  if (w == 2) {
    if (lds) SGM_ILU_BS(2, true); else SGM_ILU_BS(2, false);
  } else if (w == 4) {
    if (lds) SGM_ILU_BS(4, true); else SGM_ILU_BS(4, false);
  } else {
    if (lds) SGM_ILU_BS(8, true); else SGM_ILU_BS(8, false);
  }
#undef SGM_ILU_BS
#undef SGM_ILU
  SGM_CHECK_LAUNCH();
}

}  // namespace sgm
