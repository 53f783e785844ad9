// Tall-skinny block kernels of BCGS2 + CholQR (Alg. 2 / Alg. 4) on CDNA
// matrix cores: 16x16x4 MFMA in float64 (v_mfma_f64_16x16x4f64) or float32
// (v_mfma_f32_16x16x4f32, float32 accumulation).
//
// MFMA operand layout used throughout (wave64, one 16x16 output tile):
//   A operand: lane l supplies A[m = l%16][k = l/16]
//   B operand: lane l supplies B[k = l/16][n = l%16]
//   result:    lane l holds D[m][n = l%16] in its 4 result registers j with
//              m = 4(l/16) + j for float32 and m = l/16 + 4j for float64
//              (checked on gfx950; see drow() below)
// Every contraction over the long (row) dimension is free to assign rows to
// (step, k) pairs as long as both operands use the same assignment; the
// kernels below pick assignments that turn each lane's loads into
// contiguous vectors of a column-major matrix.
//
// Reductions over rows are two-stage and deterministic: per-workgroup
// partials in a fixed order, then a fixed-order sum over workgroups.  No
// floating-point atomics, so results are bitwise reproducible.
#include "internal.h"

#include <type_traits>

namespace sgm {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  typedef d4_t type;
};
template <>
struct Vec4<float> {
  typedef f4_t type;
};

template <typename T, int N>
struct VecN {
  T v[N];
};

__device__ __forceinline__ d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 16x16 result tile held by result register j of lane group
// g = lane / 16 (the column is lane % 16).
template <typename T>
__device__ __forceinline__ int drow(int g, int j) {
  if constexpr (sizeof(T) == 8) return g + 4 * j;
  else return 4 * g + j;
}

template <typename V>
__device__ __forceinline__ V vzero() {
  V z;
  z[0] = 0;
  z[1] = 0;
  z[2] = 0;
  z[3] = 0;
  return z;
}

// Load / store MT consecutive elements (MT in {1, 2, 4}); the address is
// aligned to MT * sizeof(T) by construction (ld and row offsets are
// multiples of 64 and MT).
template <typename T, int MT>
__device__ __forceinline__ void load_rows(const T* p, T (&out)[MT]) {
  if constexpr (MT == 4) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 v = *reinterpret_cast<const v4*>(p);
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
  } else if constexpr (MT == 2) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 v = *reinterpret_cast<const v2*>(p);
    out[0] = v[0]; out[1] = v[1];
  } else {
    out[0] = p[0];
  }
}
template <typename T, int MT>
__device__ __forceinline__ void store_rows(T* p, const T (&in)[MT]) {
  if constexpr (MT == 4) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 v;
    v[0] = in[0]; v[1] = in[1]; v[2] = in[2]; v[3] = in[3];
    *reinterpret_cast<v4*>(p) = v;
  } else if constexpr (MT == 2) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v[0] = in[0]; v[1] = in[1];
    *reinterpret_cast<v2*>(p) = v;
  } else {
    p[0] = in[0];
  }
}

constexpr int kBlock = 256;  // 4 wavefronts per workgroup

// ------------------------------------------------------------- A^T B
// C = Q(:, a0:a0+ma)^T Q(:, b0:b0+nb) over 16-row batches of Q.
// The output is cut into wave tiles of MT x NT 16x16 MFMA tiles.  A
// workgroup covers WT consecutive wave tiles over one row chunk: wavefront
// w takes wave tile w % WT and every (4/WT)-th batch of the chunk starting
// at batch w / WT (its row phase); with WT < 4 the row phases are summed
// through LDS in a fixed order.  Spreading the tiles over the wavefronts
// keeps the registers per wavefront low (4 float64 or 8 float32 tiles), so
// several workgroups share a CU and many batches are in flight; the A
// columns of different tiles are read once, the B columns they share come
// from L2.
// Grid: 1-D, chunks * ngroups workgroups (chunks a multiple of 8).
// XCD-aware decode: workgroup id -> (xcd = id % 8, slot = id / 8); the
// ngroups tile groups of one row chunk get consecutive slots on the same
// XCD and share its L2.
// Lane (g = l/16, c = l%16) loads rows 4g..4g+3 of one column as a
// 4-vector, and MFMA step t pairs row 4g + t of A with the same row of B.
// A 16-row batch never straddles a row panel, so one row offset per batch
// serves every column.
// SYM (a Gram matrix of more than 64 columns: the same columns on both
// sides): only the 16x16 tiles on and above the diagonal are formed and
// stored; the reduction mirrors the rest.  A compile-time switch: as a
// run-time test inside the unrolled MFMA loops it raised the register
// count of other tile shapes.
template <typename T, int MT, int NT, int WT, bool SYM>
__global__ __launch_bounds__(kBlock) void k_gemm_tn(
    QView<const T> Q, int a0, int ma, int b0c, int nb,
    const int* __restrict__ ncount, int64_t nbatches, int wtiles_n,
    int n_wtiles, int ngroups, int chunks, double* __restrict__ part) {
  typedef typename Vec4<T>::type V;
  constexpr int RP = (kBlock / kWave) / WT;  // row phases
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int wt = wave % WT, rp = wave / WT;
  const int id = blockIdx.x;
  const int xcd = id % 8, slot = id / 8;
  const int group = slot % ngroups;
  const int chunk = (slot / ngroups) * 8 + xcd;
  const int t = group * WT + wt;
  const int tm = t / wtiles_n, tn = t % wtiles_n;
  const int m0 = tm * 16 * MT, n0 = tn * 16 * NT;
  const int nbe = ncount ? min(nb, *ncount) : nb;
  const int64_t b0 = nbatches * chunk / chunks;
  const int64_t b1 = nbatches * (chunk + 1) / chunks;
  // M tiles of this wave tile with a valid column (0 for a spare wavefront,
  // and for a wave tile wholly below the diagonal of a symmetric product)
  const int tm0 = m0 / 16, tn0 = n0 / 16;
  const bool below = SYM && tm0 > tn0 + NT - 1;
  const int mt_live =
      t < n_wtiles && !below ? min(MT, (ma - m0 + 15) / 16) : 0;

  // per-lane column offsets; a column past the end reads column a0 / b0c
  int64_t oa[MT], ob[NT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int c = m0 + i * 16 + c16;
    oa[i] = (int64_t)(a0 + (c < ma ? c : 0)) * Q.cstride + 4 * g;
  }
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const int c = n0 + i * 16 + c16;
    ob[i] = (int64_t)(b0c + (c < nbe ? c : 0)) * Q.cstride + 4 * g;
  }
  V acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = vzero<V>();

  // Register double buffering: the loads of the next batch are in flight
  // while the MFMAs of the current one run.  Loads are unconditional: a
  // column past the end reads a valid column instead; it only feeds output
  // rows that are never stored or output columns that are zeroed at the
  // store.
  // Register double buffering: the loads of the next batch are in flight
  // while the MFMAs of the current one run.  Loads are unconditional: a
  // column past the end reads a valid column instead; it only feeds output
  // rows that are never stored or output columns that are zeroed at the
  // store.  (A ping-pong of two register sets measured 5% slower here.)
  V af[MT], bf[NT], an[MT], bn[NT];
  auto load = [&](int64_t bt, V (&a)[MT], V (&b)[NT]) {
    const T* rb = Q.base + Q.row_off(bt * 16);
#pragma unroll
    for (int i = 0; i < MT; ++i) a[i] = *reinterpret_cast<const V*>(rb + oa[i]);
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = *reinterpret_cast<const V*>(rb + ob[j]);
  };
  if (mt_live > 0) {
    int64_t bt = b0 + rp;
    if (bt < b1) load(bt, af, bf);
    for (; bt < b1; bt += RP) {
      const bool more = bt + RP < b1;
      if (more) load(bt + RP, an, bn);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          if (i >= mt_live) continue;
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            if (SYM && tm0 + i > tn0 + j) continue;  // mirrored tile
            acc[i][j] = mfma(af[i][q], bf[j][q], acc[i][j]);
          }
        }
      if (more) {
#pragma unroll
        for (int i = 0; i < MT; ++i) af[i] = an[i];
#pragma unroll
        for (int j = 0; j < NT; ++j) bf[j] = bn[j];
      }
    }
  }

  // Fixed-order sum of the row phases of each wave tile through LDS: row
  // phase RP-1 first, row phase 0 adds the sum and stores.
  constexpr int NE = MT * NT * 4;
  __shared__ double red[RP > 1 ? WT * NE * kWave : 1];
  if constexpr (RP > 1) {
    for (int r = RP - 1; r >= 1; --r) {
      if (rp == r) {
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
          for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int e = (wt * NE + (i * NT + j) * 4 + q) * kWave + lane;
              double v = (double)acc[i][j][q];
              if (r < RP - 1) v += red[e];
              red[e] = v;
            }
      }
      __syncthreads();
    }
  }
  if (rp == 0 && t < n_wtiles) {
    double* out = part + (int64_t)chunk * ma * nb;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = m0 + i * 16 + drow<T>(g, q);
          const int col = n0 + j * 16 + c16;
          if (row < ma && col < nb && !(SYM && tm0 + i > tn0 + j)) {
            double v = (double)acc[i][j][q];
            if constexpr (RP > 1)
              v += red[(wt * NE + (i * NT + j) * 4 + q) * kWave + lane];
            out[(int64_t)col * ma + row] = col < nbe ? v : 0.0;
          }
        }
  }
}

// ------------------------------------------------------------- wide A^T B
// C = Q(:, a0:a0+ma)^T Q(:, b0:b0+nb) for blocks wider than 64 columns,
// where the kernel above is bound by every wavefront fetching its own
// operands (measured at 129 x 128 over 7M rows: 37-51 of the 78.6 TFLOP/s
// float64 peak).  The output is cut into blocks of 144 x 128 (9 x 8 MFMA
// tiles); a 512-thread workgroup covers one block over one row chunk.
// Each 16-row batch of the block's 144 + 128 columns is loaded once per
// workgroup into LDS, double-buffered, and wavefront w forms the nine tiles
// of output column tile w from there.  LDS holds a batch column by column
// with a stride of 17 elements, so the 16 lanes of an operand read hit
// distinct banks.  MFMA step q pairs row 4q + g of both operands (lane
// group g = lane / 16).  Columns past ma / nbe read a valid column; their
// results are not stored (rows past ma) or stored as zero (columns past
// nbe), as in the kernel above.  Grid: nblocks * chunks workgroups (chunks
// a multiple of 8), decoded XCD-aware like the kernel above.
constexpr int kWM = 9, kWN = 8;            // tiles per output block
constexpr int kWCols = 16 * (kWM + kWN);   // 272 columns per batch
constexpr int kWStride = 17;               // LDS column stride (elements)
constexpr int kWBlock = kWN * kWave;       // one wavefront per column tile

template <typename T>
__global__ __launch_bounds__(kWBlock) void k_gemm_tn_wide(
    QView<const T> Q, int a0, int ma, int b0c, int nb,
    const int* __restrict__ ncount, int64_t nbatches, int nbn, int nblk,
    int chunks, double* __restrict__ part) {
  typedef typename Vec4<T>::type V;
  constexpr int EPV = 16 / (int)sizeof(T);  // elements per 16-byte load
  constexpr int VPC = 16 / EPV;             // loads per 16-row column batch
  constexpr int NV = kWCols * VPC;          // loads per batch
  constexpr int NVT = (NV + kWBlock - 1) / kWBlock;
  constexpr int LBUF = kWCols * kWStride;   // elements per LDS buffer
  typedef T vec_t __attribute__((ext_vector_type(EPV)));
  extern __shared__ char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int id = blockIdx.x;
  const int xcd = id % 8, slot = id / 8;
  const int blk = slot % nblk;
  const int chunk = (slot / nblk) * 8 + xcd;
  const int m0 = (blk / nbn) * 16 * kWM, n0 = (blk % nbn) * 16 * kWN;
  const int nbe = ncount ? min(nb, *ncount) : nb;
  const int64_t bt0 = nbatches * chunk / chunks;
  const int64_t bt1 = nbatches * (chunk + 1) / chunks;

  // column offset in Q of batch column `col` (A columns, then B columns)
  auto qcol = [&](int col) -> int64_t {
    int c;
    if (col < 16 * kWM) {
      c = m0 + col;
      c = a0 + (c < ma ? c : 0);
    } else {
      c = n0 + col - 16 * kWM;
      c = b0c + (c < nbe ? c : 0);
    }
    return (int64_t)c * Q.cstride;
  };
  vec_t stage[NVT];
  auto gload = [&](int64_t bt) {
    const T* rb = Q.base + Q.row_off(bt * 16);
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      const int e = threadIdx.x + kWBlock * q;
      if (e < NV)
        stage[q] = *reinterpret_cast<const vec_t*>(rb + qcol(e / VPC) +
                                                   (e % VPC) * EPV);
    }
  };
  auto lstore = [&](int buf) {
    T* L = lds + buf * LBUF;
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      const int e = threadIdx.x + kWBlock * q;
      if (e < NV) {
        T* d = L + (e / VPC) * kWStride + (e % VPC) * EPV;
#pragma unroll
        for (int u = 0; u < EPV; ++u) d[u] = stage[q][u];
      }
    }
  };

  V acc[kWM];
#pragma unroll
  for (int i = 0; i < kWM; ++i) acc[i] = vzero<V>();
  int buf = 0;
  if (bt0 < bt1) {
    gload(bt0);
    lstore(0);
  }
  __syncthreads();
  // (a ring of three register stages, as in the wide Gram below, measured
  // slower here: 41.8 against 40.2 ms at 201 x 200 over 16.8M rows)
  for (int64_t bt = bt0; bt < bt1; ++bt) {
    const bool more = bt + 1 < bt1;
    if (more) gload(bt + 1);
    const T* L = lds + buf * LBUF;
    const T* Lb = L + (16 * kWM + wave * 16 + c16) * kWStride + g;
    const T* La = L + c16 * kWStride + g;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T bv = Lb[4 * q];
#pragma unroll
      for (int i = 0; i < kWM; ++i)
        acc[i] = mfma(La[i * 16 * kWStride + 4 * q], bv, acc[i]);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* out = part + (int64_t)chunk * ma * nb;
  const int col = n0 + wave * 16 + c16;
#pragma unroll
  for (int i = 0; i < kWM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + i * 16 + drow<T>(g, r);
      if (row < ma && col < nb)
        out[(int64_t)col * ma + row] = col < nbe ? (double)acc[i][r] : 0.0;
    }
}

// ------------------------------------------------------------- tall A^T B
// C = Q(:, a0:a0+ma)^T Q(:, b0:b0+nb) for 145 to 208 rows (ma) and more than
// 96 columns, not a Gram matrix: the 144 x 128 blocks above would compute
// 288 x 256 for 201 x 200 (55% of it used) and read each column about 2.7
// times.  Here a workgroup covers all ma rows (13 tiles) and at most 112
// columns (7 tiles): each 16-row batch of those 208 + 112 columns is
// loaded into LDS once, and sixteen wavefronts take contiguous runs of at
// most 6 of the block's 91 tiles in column order (the B operand is read
// once per column of a run), as in the wide Gram.  Columns past ma / nbe
// read a valid column; their results are not stored (rows past ma) or
// stored as zero (columns past nbe).  Grid: nblk * chunks workgroups
// (chunks a multiple of 8), decoded XCD-aware like the kernel above.
constexpr int kRM = 13, kRN = 7;           // tiles per output block
constexpr int kRCols = 16 * (kRM + kRN);   // 320 columns per batch
constexpr int kRBlock = 1024;
constexpr int kRWaves = kRBlock / kWave;
constexpr int kRTiles = (kRM * kRN + kRWaves - 1) / kRWaves;

template <typename T>
__global__ __launch_bounds__(kRBlock) void k_gemm_tn_tall(
    QView<const T> Q, int a0, int ma, int b0c, int nb,
    const int* __restrict__ ncount, int64_t nbatches, int nblk, int chunks,
    double* __restrict__ part) {
  typedef typename Vec4<T>::type V;
  constexpr int EPV = 16 / (int)sizeof(T);  // elements per 16-byte load
  constexpr int VPC = 16 / EPV;             // loads per 16-row column batch
  constexpr int NV = kRCols * VPC;          // loads per batch
  constexpr int NVT = (NV + kRBlock - 1) / kRBlock;
  constexpr int LBUF = kRCols * kWStride;   // elements per LDS buffer
  typedef T vec_t __attribute__((ext_vector_type(EPV)));
  extern __shared__ char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int id = blockIdx.x;
  const int xcd = id % 8, slot = id / 8;
  const int blk = slot % nblk;
  const int chunk = (slot / nblk) * 8 + xcd;
  const int n0 = blk * 16 * kRN;
  const int nbe = ncount ? min(nb, *ncount) : nb;
  const int nta = (ma + 15) / 16;                       // <= kRM
  const int ntb = min(kRN, (nb - n0 + 15) / 16);        // this block's
  const int64_t bt0 = nbatches * chunk / chunks;
  const int64_t bt1 = nbatches * (chunk + 1) / chunks;
  // this wavefront's tiles (row tile, column tile), column-major order
  const int T_all = nta * ntb;
  const int t0 = T_all * wave / kRWaves, t1 = T_all * (wave + 1) / kRWaves;
  const int cnt = t1 - t0;
  int tr[kRTiles], tc[kRTiles];
#pragma unroll
  for (int u = 0; u < kRTiles; ++u) {
    tr[u] = (t0 + u) % nta;
    tc[u] = (t0 + u) / nta;
  }
  // column offset in Q of batch column `col` (A columns, then B columns)
  auto qcol = [&](int col) -> int64_t {
    int c;
    if (col < 16 * kRM) {
      c = a0 + (col < ma ? col : 0);
    } else {
      const int cb = n0 + col - 16 * kRM;
      c = b0c + (cb < nbe ? cb : 0);
    }
    return (int64_t)c * Q.cstride;
  };
  // three register stages in a ring: the loads of batch b + 1 go out two
  // batches before b + 1 is stored to LDS
  vec_t sA[NVT], sB[NVT], sC[NVT];
  auto gload = [&](int64_t bt, vec_t (&stg)[NVT]) {
    const T* rb = Q.base + Q.row_off(bt * 16);
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      const int e = threadIdx.x + kRBlock * q;
      if (e < NV)
        stg[q] = *reinterpret_cast<const vec_t*>(rb + qcol(e / VPC) +
                                                 (e % VPC) * EPV);
    }
  };
  auto lstore = [&](int buf, const vec_t (&stg)[NVT]) {
    T* L = lds + buf * LBUF;
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      const int e = threadIdx.x + kRBlock * q;
      if (e < NV) {
        T* d = L + (e / VPC) * kWStride + (e % VPC) * EPV;
#pragma unroll
        for (int u = 0; u < EPV; ++u) d[u] = stg[q][u];
      }
    }
  };
  V acc[kRTiles];
#pragma unroll
  for (int u = 0; u < kRTiles; ++u) acc[u] = vzero<V>();
  auto compute = [&](int buf) {
    const T* L = lds + buf * LBUF + c16 * kWStride + g;
    const T* Lb = L + 16 * kRM * kWStride;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int cur = -1;
      T bv = 0;
#pragma unroll
      for (int u = 0; u < kRTiles; ++u) {
        if (u < cnt) {
          if (tc[u] != cur) {
            cur = tc[u];
            bv = Lb[cur * 16 * kWStride + 4 * q];
          }
          acc[u] = mfma(L[tr[u] * 16 * kWStride + 4 * q], bv, acc[u]);
        }
      }
    }
  };
  int buf = 0;
  auto step = [&](int64_t b, const vec_t (&nxt)[NVT], vec_t (&fre)[NVT]) {
    if (b >= bt1) return;
    compute(buf);
    if (b + 1 < bt1) lstore(buf ^ 1, nxt);
    if (b + 3 < bt1) gload(b + 3, fre);
    __syncthreads();
    buf ^= 1;
  };
  if (bt0 < bt1) {
    gload(bt0, sA);
    lstore(0, sA);
  }
  if (bt0 + 1 < bt1) gload(bt0 + 1, sB);
  if (bt0 + 2 < bt1) gload(bt0 + 2, sC);
  __syncthreads();
  for (int64_t bt = bt0; bt < bt1; bt += 3) {
    step(bt, sB, sA);
    step(bt + 1, sC, sB);
    step(bt + 2, sA, sC);
  }
  double* out = part + (int64_t)chunk * ma * nb;
#pragma unroll
  for (int u = 0; u < kRTiles; ++u) {
    if (u < cnt) {
      const int col = n0 + tc[u] * 16 + c16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tr[u] * 16 + drow<T>(g, r);
        if (row < ma && col < nb)
          out[(int64_t)col * ma + row] =
              col < nbe ? (double)acc[u][r] : 0.0;
      }
    }
  }
}

// ------------------------------------------------------------- wide Gram
// G = Q(:, b0:b0+nb)^T Q(:, b0:b0+nb) for Gram matrices of 65 to 256
// columns.  One 1024-thread workgroup per row chunk loads each 16-row batch
// of all nb columns into LDS once (double-buffered, column stride ROWS + 1), and
// the sixteen wavefronts form the nt (nt + 1) / 2 tiles on and above the
// diagonal (nt = 16 ceil(nb / 16)) from there: wavefront w takes the
// contiguous run [T w / 16, T (w + 1) / 16) of them in column order, so
// consecutive tiles mostly share their B operand, which is read once per
// column.  Sixteen wavefronts of at most 9 tiles fit four to a SIMD (eight
// of 17 fitted two): 20.5 -> 15.9 ms for 200 columns over 16.8M rows, and
// 32-row batches with at most 7 tiles (up to 224 columns) 15.6 -> 14.7 ms.
// The reduction mirrors the lower tiles.  Columns past nb read a
// valid column (their results are not stored); columns past *ncount give
// zero (as in the kernels above).  Grid: chunks workgroups, each a
// contiguous range of batches.
constexpr int kGBlock = 1024;            // 16 wavefronts
constexpr int kGWaves = kGBlock / kWave;
// most tiles per wavefront: 136 tiles on and above the diagonal at nb = 256
constexpr int kGTiles = (136 + kGWaves - 1) / kGWaves;
constexpr int kGMaxCols = 256;
// Rows per batch (ROWS) and the LDS column stride ROWS + 1 (odd: no bank
// conflicts between the lanes' columns).  32-row batches give each barrier
// and LDS store round eight MFMA k-steps instead of four; with nine tiles
// per wavefront the float64 kernel then needs more than 128 registers, so
// that case keeps 16-row batches.

template <typename T, int TILES, int ROWS>
__global__ __launch_bounds__(kGBlock) void k_gram_wide(
    QView<const T> Q, int b0c, int nb, const int* __restrict__ ncount,
    int64_t nbatches, int chunks, double* __restrict__ part) {
  typedef typename Vec4<T>::type V;
  constexpr int EPV = 16 / (int)sizeof(T);  // elements per 16-byte load
  constexpr int VPC = ROWS / EPV;         // loads per column of a batch
  constexpr int NVT = (kGMaxCols * VPC + kGBlock - 1) / kGBlock;
  typedef T vec_t __attribute__((ext_vector_type(EPV)));
  extern __shared__ char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int nt = (nb + 15) / 16;
  const int ncols = nt * 16;
  const int NV = ncols * VPC;               // loads per batch
  const int LBUF = ncols * (ROWS + 1);        // elements per LDS buffer
  const int nbe = ncount ? min(nb, *ncount) : nb;
  const int chunk = blockIdx.x;
  const int64_t bt0 = nbatches * chunk / chunks;
  const int64_t bt1 = nbatches * (chunk + 1) / chunks;
  // this wavefront's tiles (row tile, column tile), column-major order of
  // the upper triangle (wavefront-uniform)
  const int T_all = nt * (nt + 1) / 2;
  const int t0 = T_all * wave / kGWaves, t1 = T_all * (wave + 1) / kGWaves;
  int tr[TILES], tc[TILES];
  {
    int c = 0, base = 0;  // tiles of columns < c: base = c (c + 1) / 2
    while (base + c + 1 <= t0) {
      base += c + 1;
      ++c;
    }
    int r = t0 - base;
#pragma unroll
    for (int u = 0; u < TILES; ++u) {
      tr[u] = r;
      tc[u] = c;
      if (++r > c) {
        ++c;
        r = 0;
      }
    }
  }
  const int cnt = t1 - t0;

  // two register stages: the loads of batch b + 2 go out while batch b is
  // formed, and are stored to LDS after it, so their latency is covered by
  // the MFMA work of a whole batch
  vec_t sA[NVT], sB[NVT];
  auto gload = [&](int64_t bt, vec_t (&stg)[NVT]) {
    const T* rb = Q.base + Q.row_off(bt * ROWS);
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      const int e = threadIdx.x + kGBlock * q;
      if (e < NV) {
        const int col = e / VPC;
        const int c = b0c + (col < nb ? col : 0);
        stg[q] = *reinterpret_cast<const vec_t*>(
            rb + (int64_t)c * Q.cstride + (e % VPC) * EPV);
      }
    }
  };
  auto lstore = [&](int buf, const vec_t (&stg)[NVT]) {
    T* L = lds + buf * LBUF;
#pragma unroll
    for (int q = 0; q < NVT; ++q) {
      const int e = threadIdx.x + kGBlock * q;
      if (e < NV) {
        T* d = L + (e / VPC) * (ROWS + 1) + (e % VPC) * EPV;
#pragma unroll
        for (int u = 0; u < EPV; ++u) d[u] = stg[q][u];
      }
    }
  };

  V acc[TILES];
#pragma unroll
  for (int u = 0; u < TILES; ++u) acc[u] = vzero<V>();
  auto compute = [&](int buf) {
    const T* L = lds + buf * LBUF + c16 * (ROWS + 1) + g;
#pragma unroll
    for (int q = 0; q < ROWS / 4; ++q) {
      int cur = -1;
      T bv = 0;
#pragma unroll
      for (int u = 0; u < TILES; ++u) {
        if (u < cnt) {
          if (tc[u] != cur) {
            cur = tc[u];
            bv = L[cur * 16 * (ROWS + 1) + 4 * q];
          }
          acc[u] = mfma(L[tr[u] * 16 * (ROWS + 1) + 4 * q], bv, acc[u]);
        }
      }
    }
  };
  int buf = 0;
  // batch b: compute from LDS, store batch b + 1 (registers `nxt`) to the
  // other LDS buffer, load batch b + 2 into the registers `fre` that held
  // batch b (storing and loading before the MFMA work measured slower: the
  // store then waits for loads issued only one batch earlier)
  auto step = [&](int64_t b, const vec_t (&nxt)[NVT], vec_t (&fre)[NVT]) {
    if (b >= bt1) return;
    compute(buf);
    if (b + 1 < bt1) lstore(buf ^ 1, nxt);
    if (b + 2 < bt1) gload(b + 2, fre);
    __syncthreads();
    buf ^= 1;
  };
  if (bt0 < bt1) {
    gload(bt0, sA);
    lstore(0, sA);
  }
  if (bt0 + 1 < bt1) gload(bt0 + 1, sB);
  __syncthreads();
  for (int64_t bt = bt0; bt < bt1; bt += 2) {
    step(bt, sB, sA);
    step(bt + 1, sA, sB);
  }
  double* out = part + (int64_t)chunk * nb * nb;
#pragma unroll
  for (int u = 0; u < TILES; ++u) {
    if (u < cnt) {
      const int col = tc[u] * 16 + c16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tr[u] * 16 + drow<T>(g, r);
        if (row < nb && col < nb)
          out[(int64_t)col * nb + row] =
              (col < nbe && row < nbe) ? (double)acc[u][r] : 0.0;
      }
    }
  }
}

// Fixed-order sums over the chunks of partial results.  A workgroup of
// 1024 threads takes kRedOut consecutive outputs: thread t sums output
// t % kRedOut over the chunks c = g, g + kRedGroups, ... (g = t / kRedOut)
// with up to 16 loads in flight (one round for up to 1024 chunks; each
// load instruction reads kRedOut consecutive doubles per chunk), then the
// kRedGroups sums meet in a fixed LDS tree.  Deterministic.  (One output
// per lane and 16 chunk groups per workgroup took four dependent load
// rounds at 512 chunks and a sixteenth of the workgroups.)
constexpr int kRedThreads = 1024;
constexpr int kRedOut = 16;
constexpr int kRedGroups = kRedThreads / kRedOut;
constexpr int kRedBatch = 16;

// Sum of part[c * stride + src] over the thread's chunks, in chunk order.
__device__ __forceinline__ double chunk_sum(const double* __restrict__ part,
                                            int64_t nchunks, int64_t stride,
                                            int64_t src, int g) {
  double s = 0.0;
  for (int64_t c = g; c < nchunks; c += kRedBatch * kRedGroups) {
    double a[kRedBatch];
#pragma unroll
    for (int q = 0; q < kRedBatch; ++q) {
      const int64_t cq = c + (int64_t)q * kRedGroups;
      a[q] = cq < nchunks ? part[cq * stride + src] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kRedBatch; ++q) s += a[q];
  }
  return s;
}

// red[t] holds thread t's sum; afterwards red[o] (o < kRedOut) holds the
// total of output o, added over the groups in a fixed tree.
__device__ __forceinline__ void group_tree(double* red) {
  const int g = threadIdx.x / kRedOut;
  __syncthreads();
#pragma unroll
  for (int h = kRedGroups / 2; h > 0; h >>= 1) {
    if (g < h) red[threadIdx.x] += red[threadIdx.x + h * kRedOut];
    __syncthreads();
  }
}

// C(i, j) = sum over chunks of part[c][j * ma + i]; with sym, entries below
// the diagonal 16x16 tiles are read from the mirrored upper entry.
__global__ __launch_bounds__(kRedThreads) void k_reduce_chunks(
    const double* __restrict__ part, int64_t nchunks, int ma, int nb,
    double* __restrict__ C, int ldc, int sym) {
  __shared__ double red[kRedThreads];
  const int o = threadIdx.x % kRedOut, g = threadIdx.x / kRedOut;
  const int64_t e = (int64_t)blockIdx.x * kRedOut + o;
  const int64_t ne = (int64_t)ma * nb;
  const int i = (int)(e % ma), j = (int)(e / ma);
  double s = 0.0;
  if (e < ne) {
    const int64_t src =
        (sym && (i / 16) > (j / 16)) ? (int64_t)i * ma + j : e;
    s = chunk_sum(part, nchunks, ne, src, g);
  }
  red[threadIdx.x] = s;
  group_tree(red);
  if (g == 0 && e < ne) C[(int64_t)j * ldc + i] = red[o];
}

void launch_reduce(const double* part, int64_t nchunks, int ma, int nb,
                   double* C, int ldc, int sym, hipStream_t st) {
  const int64_t ne = (int64_t)ma * nb;
  hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)ceil_div(ne, kRedOut)),
                     dim3(kRedThreads), 0, st, part, nchunks, ma, nb, C, ldc,
                     sym);
  SGM_CHECK_LAUNCH();
}

// ------------------------------------------------------------- update / trsm
// One wavefront owns 16*MT consecutive rows and every column of the block.
// Tile row m of row-tile t is physical row r0 + MT*m + t, so a lane's A
// operand for the MT row tiles is one contiguous MT-vector of a column, and
// the MT results sharing a D index are contiguous rows too.
// With A = Q(:, a0:a0+ka) and B = Q(:, b0:b0+nc):
// MODE_UPDATE: B(:, 0:nc) = B - A M(0:ka, 0:nc), and (GRAM) the partial
//              Gram B^T B of the updated rows.
// MODE_TRSM:   B(:, 0:p) = B(:, 0:p) M(0:p, 0:p) in place, M upper
//              triangular (tiles below the diagonal are skipped).
// A wavefront's 16*MT rows (16, 32 or 64, aligned) lie in one row panel.
// M is staged in LDS (negated for the update) in chunks of kc rows; when it
// fits whole it is staged once per workgroup, which then walks its row
// blocks without further barriers.  Wide blocks take BLOCK = 512 or 1024
// threads, so the wavefronts of a CU share one staged copy.
enum { MODE_UPDATE = 0, MODE_TRSM = 1 };

// PACKED (MODE_TRSM only): M's upper triangle on the p accepted columns is
// staged once per workgroup packed row by row (row k holds columns
// k .. p-1 at k p - k (k - 1) / 2), so a triangular factor of up to 200
// float64 columns fits in LDS whole instead of being re-staged in chunks
// for every row block.
template <typename T, int NT, int MT, int MODE, bool GRAM, int BLOCK = kBlock,
          bool PACKED = false>
__global__ __launch_bounds__(BLOCK) void k_update(
    QView<T> Q, int a0, int ka, int b0c, int nc,
    const double* __restrict__ M, int ldm, const int* __restrict__ ncount,
    int64_t nrows, int kc, double* __restrict__ part, int nc_off = 0) {
  typedef typename Vec4<T>::type V;
  extern __shared__ char smem_raw[];
  T* Ms = reinterpret_cast<T*>(smem_raw);
  constexpr int W16 = NT * 16;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  int nce = nc;
  // a column group starting nc_off columns into the block keeps the
  // block's accepted columns: *ncount - nc_off of its own
  if (ncount) nce = max(0, min(nc, *ncount - nc_off));
  int kae = ka;
  if (MODE == MODE_TRSM) kae = nce;
  const int ka4 = (kae + 3) & ~3;
  const bool single = PACKED || ka4 <= kc;
  const int64_t rows_per_wave = 16 * MT;
  const int64_t rows_per_block = rows_per_wave * (BLOCK / kWave);
  const int64_t nblocks = (nrows + rows_per_block - 1) / rows_per_block;
  // wide blocks of one 16-row tile per wavefront in 512-thread workgroups
  // (256 registers a lane): loads two groups ahead
  constexpr bool DEEP = MT == 1 && NT >= 8 && !GRAM && BLOCK <= 512;

  auto stage = [&](int k0) {
    if constexpr (PACKED) {
      for (int e = threadIdx.x; e < nce * nce; e += BLOCK) {
        const int k = e / nce, c = e % nce;
        if (c >= k)
          Ms[k * nce - k * (k - 1) / 2 + (c - k)] =
              (T)M[(int64_t)c * ldm + k];
      }
      return;
    }
    for (int e = threadIdx.x; e < kc * W16; e += BLOCK) {
      const int kk = e / W16, cc = e % W16;
      const int k = k0 + kk;
      double v = 0.0;
      if (k < kae && cc < nce) {
        v = M[(int64_t)cc * ldm + k];
        if (MODE == MODE_UPDATE) v = -v;
      }
      Ms[e] = (T)v;
    }
  };

  constexpr int NG = GRAM ? NT * (NT + 1) / 2 : 1;
  V gacc[NG];
#pragma unroll
  for (int t = 0; t < NG; ++t) gacc[t] = vzero<V>();

  if (single) {
    stage(0);
    __syncthreads();
  }
  for (int64_t rb = blockIdx.x; rb < nblocks; rb += gridDim.x) {
    const int64_t r0 = rb * rows_per_block + wave * rows_per_wave;
    const bool active = r0 < nrows;
    T* const rbase = Q.base + Q.row_off(r0);
    T* const B = rbase + (int64_t)b0c * Q.cstride;
    const int64_t cs = Q.cstride;
    V acc[MT][NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int c = j * 16 + c16;
      if (MODE == MODE_UPDATE && active && c < nce) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T v[MT];
          load_rows<T, MT>(B + (int64_t)c * cs + MT * drow<T>(g, q), v);
#pragma unroll
          for (int t = 0; t < MT; ++t) acc[t][j][q] = v[t];
        }
      } else {
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t][j] = vzero<V>();
      }
    }
    for (int k0 = 0; k0 < ka4; k0 += kc) {
      if (!single) {
        __syncthreads();
        stage(k0);
        __syncthreads();
      }
      const int kend = min(kc, ka4 - k0);
      if (active) {
        const T* base = rbase +
                        (int64_t)(MODE == MODE_TRSM ? b0c : a0) * cs +
                        MT * c16;
        auto kstep = [&](int kk, const T (&a)[MT]) {
          if constexpr (PACKED && BLOCK <= 512) {
            // row kp of the packed triangle, column c at prow[c].  The
            // k-step's four rows share one 16-column tile for their
            // diagonal (jd), and only the last k-step can hold rows past
            // the accepted columns: only those reads are masked (zero left
            // of the diagonal and on rows past nce); the others are plain
            // LDS reads at a constant offset.  A column past nce may read
            // another row's value or the padding after the triangle; it
            // only reaches output columns that are never stored.
            // All NT reads go out together, unconditionally (the tiles
            // left of the diagonal read entries of earlier rows, rows past
            // nce the padding after the triangle: all inside the array),
            // then one wait, then the masks as selects and the MFMAs (a
            // masked read per tile made every tile wait for its own LDS
            // round trip).
            const int kp = k0 + kk + g;
            const T* prow = Ms + (kp * nce - kp * (kp - 1) / 2) - kp + c16;
            const int kb = k0 + kk;
            const int jd = kb >> 4;
            const bool tail = kb + 4 > nce;
            T bv[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) bv[j] = prow[j * 16];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
              if (kb >= (j + 1) * 16) continue;
              T b = bv[j];
              if (j == jd || tail)
                b = (j * 16 + c16 >= kp && kp < nce) ? b : (T)0;
#pragma unroll
              for (int t = 0; t < MT; ++t)
                acc[t][j] = mfma(a[t], b, acc[t][j]);
            }
          } else {
            const T* mrow = Ms + (kk + g) * W16 + c16;
            // packed: row k of the triangle (zero left of the diagonal and
            // past the accepted columns)
            const int kp = k0 + kk + g;
            const T* prow = Ms + (kp * nce - kp * (kp - 1) / 2) - kp;
            // the staged rows' reads go out together before the MFMAs (a
            // read after each tile's triangle test waited per tile), where
            // the registers allow (1024-thread variants of more than 8
            // tiles would spill)
            constexpr bool BATCH = !PACKED && (BLOCK <= 512 || NT <= 8);
            T bs[NT];
            if constexpr (BATCH) {
#pragma unroll
              for (int j = 0; j < NT; ++j) bs[j] = mrow[j * 16];
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
              if (MODE == MODE_TRSM && (k0 + kk) >= (j + 1) * 16) continue;
              T bv;
              if constexpr (PACKED) {
                const int c = j * 16 + c16;
                bv = (c >= kp && c < nce && kp < nce) ? prow[c] : (T)0;
              } else if constexpr (BATCH) {
                bv = bs[j];
              } else {
                bv = mrow[j * 16];
              }
#pragma unroll
              for (int t = 0; t < MT; ++t)
                acc[t][j] = mfma(a[t], bv, acc[t][j]);
            }
          }
        };
        // unconditional loads: a column past the end reads column 0, whose
        // staged M row is zero, so no branch or select splits the
        // outstanding loads
        auto kload = [&](int kk, T (&a)[MT]) {
          const int k = k0 + kk + g;
          load_rows<T, MT>(base + (int64_t)(k < kae ? k : 0) * cs, a);
        };
        // four k-steps per group; the next group's loads are issued before
        // the current group's MFMAs, into the other of two register sets
        // (ping-pong, no copies: a copy of a register still being loaded
        // would make every group wait for its successor's loads).  The
        // prefetch past the last group reads column 0 and is not used.
        const int kend16 = kend & ~15;
        if (DEEP && kend16 > 0) {
          // three register sets: the loads of the group two ahead are in
          // flight while a group is multiplied (a wavefront of one 16-row
          // tile per column keeps too few bytes in flight with two)
          T x0[MT], x1[MT], x2[MT], x3[MT], y0[MT], y1[MT], y2[MT], y3[MT],
              z0[MT], z1[MT], z2[MT], z3[MT];
          kload(0, x0);
          kload(4, x1);
          kload(8, x2);
          kload(12, x3);
          kload(16, y0);
          kload(20, y1);
          kload(24, y2);
          kload(28, y3);
          for (int kg = 0; kg < kend16; kg += 48) {
            kload(kg + 32, z0);
            kload(kg + 36, z1);
            kload(kg + 40, z2);
            kload(kg + 44, z3);
            __builtin_amdgcn_sched_barrier(0);
            kstep(kg, x0);
            kstep(kg + 4, x1);
            kstep(kg + 8, x2);
            kstep(kg + 12, x3);
            if (kg + 16 >= kend16) break;
            kload(kg + 48, x0);
            kload(kg + 52, x1);
            kload(kg + 56, x2);
            kload(kg + 60, x3);
            __builtin_amdgcn_sched_barrier(0);
            kstep(kg + 16, y0);
            kstep(kg + 20, y1);
            kstep(kg + 24, y2);
            kstep(kg + 28, y3);
            if (kg + 32 >= kend16) break;
            kload(kg + 64, y0);
            kload(kg + 68, y1);
            kload(kg + 72, y2);
            kload(kg + 76, y3);
            __builtin_amdgcn_sched_barrier(0);
            kstep(kg + 32, z0);
            kstep(kg + 36, z1);
            kstep(kg + 40, z2);
            kstep(kg + 44, z3);
          }
        } else if (kend16 > 0) {
          T x0[MT], x1[MT], x2[MT], x3[MT], y0[MT], y1[MT], y2[MT], y3[MT];
          kload(0, x0);
          kload(4, x1);
          kload(8, x2);
          kload(12, x3);
          for (int kg = 0; kg < kend16; kg += 32) {
            kload(kg + 16, y0);
            kload(kg + 20, y1);
            kload(kg + 24, y2);
            kload(kg + 28, y3);
            // keep the prefetch ahead of the MFMAs (the scheduler would
            // otherwise sink each load down to its first use)
            __builtin_amdgcn_sched_barrier(0);
            kstep(kg, x0);
            kstep(kg + 4, x1);
            kstep(kg + 8, x2);
            kstep(kg + 12, x3);
            if (kg + 16 >= kend16) break;
            kload(kg + 32, x0);
            kload(kg + 36, x1);
            kload(kg + 40, x2);
            kload(kg + 44, x3);
            __builtin_amdgcn_sched_barrier(0);
            kstep(kg + 16, y0);
            kstep(kg + 20, y1);
            kstep(kg + 24, y2);
            kstep(kg + 28, y3);
          }
        }
        for (int kk = kend16; kk < kend; kk += 4) {
          T a0[MT];
          kload(kk, a0);
          kstep(kk, a0);
        }
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int c = j * 16 + c16;
        if (c < nce) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            T v[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t) v[t] = acc[t][j][q];
            store_rows<T, MT>(B + (int64_t)c * cs + MT * drow<T>(g, q), v);
          }
        }
      }
      if constexpr (GRAM) {
        int tix = 0;
#pragma unroll
        for (int j1 = 0; j1 < NT; ++j1)
#pragma unroll
          for (int j2 = j1; j2 < NT; ++j2) {
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                gacc[tix] = mfma(acc[t][j1][q], acc[t][j2][q], gacc[tix]);
            ++tix;
          }
      }
    }
  }
  if constexpr (GRAM) {
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem_raw);
    constexpr int NE = NG * 4;
    for (int w = BLOCK / kWave - 1; w >= 1; --w) {
      if (wave == w) {
#pragma unroll
        for (int t = 0; t < NG; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = (t * 4 + q) * kWave + lane;
            double v = (double)gacc[t][q];
            if (w < BLOCK / kWave - 1) v += red[e];
            red[e] = v;
          }
      }
      __syncthreads();
    }
    if (wave == 0) {
      double* out = part + (int64_t)blockIdx.x * nc * nc;
      int tix = 0;
#pragma unroll
      for (int j1 = 0; j1 < NT; ++j1)
#pragma unroll
        for (int j2 = j1; j2 < NT; ++j2) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = (tix * 4 + q) * kWave + lane;
            const int row = j1 * 16 + drow<T>(g, q);
            const int col = j2 * 16 + c16;
            if (row < nc && col < nc)
              out[(int64_t)col * nc + row] = (double)gacc[tix][q] + red[e];
          }
          ++tix;
        }
      (void)NE;
    }
  }
}

// Fused first-pass normalisation and second projection of BCGS2 (Alg. 4):
//   Q_k = V(:, 0:p) Zinv(0:p, 0:p) (stored in place, V = Q(:, b0c:b0c+nc)),
//   part[block] = Q(:, 0:ka)^T Q_k summed over the block's rows,
// with p = min(nc, *pcount).  The projection takes the values of Q_k from
// the registers the triangular product leaves them in, i.e. exactly the
// stored (rounded) values, as Alg. 4 projects the stored Q_k.  In that
// register layout, result register q of row tile t holds row
// r0 + MT * drow(g, q) + t, which is the row the projection's MFMA step
// (q, t) needs in lane group g; the matching A operand, column
// 16 i + c16 of Q at those MT rows, is one MT-vector load.
// Requires ka <= 16 * MQ (MQ column tiles of Q accumulate in registers).
template <typename T, int NT, int MT, int MQ>
__global__ __launch_bounds__(kBlock) void k_trsm_proj(
    QView<T> Q, int ka, int b0c, int nc, const double* __restrict__ Zinv,
    int ldz, const int* __restrict__ pcount, int64_t nrows,
    double* __restrict__ part) {
  typedef typename Vec4<T>::type V;
  extern __shared__ char smem_raw[];
  T* Ms = reinterpret_cast<T*>(smem_raw);
  constexpr int W16 = NT * 16;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int nce = pcount ? min(nc, *pcount) : nc;
  const int ka4 = (nce + 3) & ~3;
  const int mq_live = (ka + 15) / 16;
  const int64_t cs = Q.cstride;
  const int64_t rows_per_wave = 16 * MT;
  const int64_t rows_per_block = rows_per_wave * (kBlock / kWave);
  const int64_t nblocks = (nrows + rows_per_block - 1) / rows_per_block;
  // Zinv (upper triangular, masked to the p accepted columns) in LDS
  for (int e = threadIdx.x; e < ka4 * W16; e += kBlock) {
    const int kk = e / W16, cc = e % W16;
    Ms[e] = (T)(kk < nce && cc < nce ? Zinv[(int64_t)cc * ldz + kk] : 0.0);
  }
  __syncthreads();
  // Q column offsets of the projection's A operand (a column past ka
  // reads column 0; its rows of the result are not stored)
  int64_t oq[MQ];
#pragma unroll
  for (int i = 0; i < MQ; ++i) {
    const int c = i * 16 + c16;
    oq[i] = (int64_t)(c < ka ? c : 0) * cs;
  }
  V r2[MQ][NT];
#pragma unroll
  for (int i = 0; i < MQ; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) r2[i][j] = vzero<V>();

  for (int64_t rb = blockIdx.x; rb < nblocks; rb += gridDim.x) {
    const int64_t r0 = rb * rows_per_block + wave * rows_per_wave;
    if (r0 >= nrows || nce == 0) continue;
    T* const rbase = Q.base + Q.row_off(r0);
    T* const B = rbase + (int64_t)b0c * cs;
    // triangular product: acc = V(:, 0:p) Zinv
    V acc[MT][NT];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[t][j] = vzero<V>();
    const T* vbase = B + MT * c16;
    for (int kk = 0; kk < ka4; kk += 4) {
      const int k = kk + g;
      T a[MT];
      load_rows<T, MT>(vbase + (int64_t)(k < nce ? k : 0) * cs, a);
      const T* mrow = Ms + (kk + g) * W16 + c16;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        if (kk >= (j + 1) * 16) continue;  // below the diagonal tiles
        const T bv = mrow[j * 16];
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t][j] = mfma(a[t], bv, acc[t][j]);
      }
    }
    // store Q_k (the accepted columns)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int c = j * 16 + c16;
      if (c < nce) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T v[MT];
#pragma unroll
          for (int t = 0; t < MT; ++t) v[t] = acc[t][j][q];
          store_rows<T, MT>(B + (int64_t)c * cs + MT * drow<T>(g, q), v);
        }
      }
    }
    // projection: r2(i, j) += Q(rows, 16i + m)^T Q_k(rows, 16j + n)
#pragma unroll
    for (int i = 0; i < MQ; ++i) {
      if (i >= mq_live) continue;
      T qa[4][MT];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        load_rows<T, MT>(rbase + oq[i] + MT * drow<T>(g, q), qa[q]);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
          for (int j = 0; j < NT; ++j)
            r2[i][j] = mfma(qa[q][t], acc[t][j][q], r2[i][j]);
    }
  }
  // fixed-order sum of the four wavefronts through LDS, then one partial
  // per workgroup
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem_raw);
  constexpr int NE = MQ * NT * 4;
  for (int w = kBlock / kWave - 1; w >= 1; --w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < MQ; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int e = ((i * NT + j) * 4 + q) * kWave + lane;
            double v = (double)r2[i][j][q];
            if (w < kBlock / kWave - 1) v += red[e];
            red[e] = v;
          }
    }
    __syncthreads();
  }
  if (wave == 0) {
    double* out = part + (int64_t)blockIdx.x * ka * nc;
#pragma unroll
    for (int i = 0; i < MQ; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = ((i * NT + j) * 4 + q) * kWave + lane;
          const int row = i * 16 + drow<T>(g, q);
          const int col = j * 16 + c16;
          if (row < ka && col < nc)
            out[(int64_t)col * ka + row] = (double)r2[i][j][q] + red[e];
        }
  }
  (void)NE;
}

// Second pass of the Pythagorean BCGS2 variant, update and triangular
// solve in one pass over the block:
//   V(:, 0:p) = (V(:, 0:p) - Q(:, 0:ka) M(0:ka, 0:p)) Zinv(0:p, 0:p),
// V = Q(:, b0c : b0c+nc), p = min(nc, *pcount) (the second pass's accepted
// size; columns p.. are left as they are), Zinv upper triangular.
// The update is computed transposed, U^T = V^T - M^T Q^T: the same MFMA as
// the plain update with the operands swapped (the staged M supplies the A
// side, Q the B side, with unchanged loads), so tile acc[t][j] holds U^T
// with lane (g, c16) owning row r0 + MT * c16 + t and, in result register
// q, column 16 j + drow(g, q).  That register is the B operand of the next
// product Y^T = Zinv^T U^T for MFMA step (j, q), whose k slot g is then
// column 16 j + drow(g, q): no transpose through LDS is needed.  The
// result Y^T has the same layout, so each lane stores MT consecutive rows
// of a column.  Output tiles are formed from the last to the first: tile
// jo needs U tiles 0..jo only, so it can overwrite U tile jo.
// LDS: Zinv (W16 x W16) then the staged -M (kc x W16).
template <typename T, int NT, int MT>
__global__ __launch_bounds__(kBlock) void k_update_trsm(
    QView<T> Q, int ka, int b0c, int nc, const double* __restrict__ M,
    int ldm, const double* __restrict__ Zinv, int ldz,
    const int* __restrict__ pcount, int64_t nrows, int kc) {
  typedef typename Vec4<T>::type V;
  extern __shared__ char smem_raw[];
  constexpr int W16 = NT * 16;
  T* Zs = reinterpret_cast<T*>(smem_raw);
  T* Ms = Zs + W16 * W16;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int g = lane / 16, c16 = lane % 16;
  const int p = min(nc, *pcount);
  if (p <= 0) return;  // uniform over the grid
  const int ka4 = (ka + 3) & ~3;
  const bool single = ka4 <= kc;
  const int64_t cs = Q.cstride;
  const int64_t rows_per_wave = 16 * MT;
  const int64_t rows_per_block = rows_per_wave * (kBlock / kWave);
  const int64_t nblocks = (nrows + rows_per_block - 1) / rows_per_block;

  for (int e = threadIdx.x; e < W16 * W16; e += kBlock) {
    const int k = e / W16, c = e % W16;
    Zs[e] = (T)(k <= c && c < p ? Zinv[(int64_t)c * ldz + k] : 0.0);
  }
  auto stage = [&](int k0) {
    for (int e = threadIdx.x; e < kc * W16; e += kBlock) {
      const int kk = e / W16, cc = e % W16;
      const int k = k0 + kk;
      Ms[e] = (T)(k < ka && cc < p ? -M[(int64_t)cc * ldm + k] : 0.0);
    }
  };
  if (single) stage(0);
  __syncthreads();

  for (int64_t rb = blockIdx.x; rb < nblocks; rb += gridDim.x) {
    const int64_t r0 = rb * rows_per_block + wave * rows_per_wave;
    const bool active = r0 < nrows;
    T* const rbase = Q.base + Q.row_off(r0);
    T* const B = rbase + (int64_t)b0c * cs;
    V acc[MT][NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = j * 16 + drow<T>(g, q);
        T v[MT];
        if (active && c < p) {
          load_rows<T, MT>(B + (int64_t)c * cs + MT * c16, v);
        } else {
#pragma unroll
          for (int t = 0; t < MT; ++t) v[t] = (T)0;
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t][j][q] = v[t];
      }
    for (int k0 = 0; k0 < ka4; k0 += kc) {
      if (!single) {
        __syncthreads();
        stage(k0);
        __syncthreads();
      }
      const int kend = min(kc, ka4 - k0);
      if (active) {
        const T* base = rbase + MT * c16;
        auto kstep = [&](int kk, const T (&a)[MT]) {
          const T* mrow = Ms + (kk + g) * W16 + c16;
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const T av = mrow[j * 16];
#pragma unroll
            for (int t = 0; t < MT; ++t) acc[t][j] = mfma(av, a[t], acc[t][j]);
          }
        };
        // a column past the end reads column 0, whose staged M row is zero
        auto kload = [&](int kk, T (&a)[MT]) {
          const int k = k0 + kk + g;
          load_rows<T, MT>(base + (int64_t)(k < ka ? k : 0) * cs, a);
        };
        int kk = 0;
        const int kend16 = kend & ~15;
        if (kend16 > 0) {
          T a0[MT], a1[MT], a2[MT], a3[MT];
          kload(0, a0);
          kload(4, a1);
          kload(8, a2);
          kload(12, a3);
          for (; kk < kend16; kk += 16) {
            T n0[MT], n1[MT], n2[MT], n3[MT];
            const bool more = kk + 16 < kend16;
            if (more) {
              kload(kk + 16, n0);
              kload(kk + 20, n1);
              kload(kk + 24, n2);
              kload(kk + 28, n3);
            }
            kstep(kk, a0);
            kstep(kk + 4, a1);
            kstep(kk + 8, a2);
            kstep(kk + 12, a3);
            if (more) {
#pragma unroll
              for (int t = 0; t < MT; ++t) {
                a0[t] = n0[t];
                a1[t] = n1[t];
                a2[t] = n2[t];
                a3[t] = n3[t];
              }
            }
          }
        }
        for (; kk < kend; kk += 4) {
          T a0[MT];
          kload(kk, a0);
          kstep(kk, a0);
        }
      }
    }
    if (active) {
      // Y^T = Zinv^T U^T, output tiles from the last to the first
#pragma unroll
      for (int jo = NT - 1; jo >= 0; --jo) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          V o = vzero<V>();
#pragma unroll
          for (int jt = 0; jt <= jo; ++jt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const T zv = Zs[(jt * 16 + drow<T>(g, q)) * W16 + jo * 16 + c16];
              o = mfma(zv, acc[t][jt][q], o);
            }
          acc[t][jo] = o;
        }
      }
#pragma unroll
      for (int jo = 0; jo < NT; ++jo)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = jo * 16 + drow<T>(g, q);
          if (c < p) {
            T v[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t) v[t] = acc[t][jo][q];
            store_rows<T, MT>(B + (int64_t)c * cs + MT * c16, v);
          }
        }
    }
  }
}

// Second Gram of the Pythagorean BCGS2 variant (float64):
//   G2(a, b) = Gk(a, b) - sum_k R2(k, a) R2(k, b),  a, b < p1 = *pcount,
// zero outside, from C = [R2; Gk] ((ka + nc) x nc, ld ldc; Gk is read on
// and above the diagonal).  One workgroup per column b: R2(:, b) is staged
// in LDS; each wavefront takes columns a, its lanes split k (lane l sums
// k = l, l + 64, ...), then a fixed xor tree.  The sums for (a, b) and
// (b, a) multiply the same pairs in the same order, so G2 is exactly
// symmetric.  Deterministic.
__global__ __launch_bounds__(256) void k_pyth_gram(
    const double* __restrict__ C, int ldc, int ka, int nc,
    const int* __restrict__ pcount, double* __restrict__ G2, int ldg) {
  extern __shared__ char smem_raw[];
  double* rb = reinterpret_cast<double*>(smem_raw);
  const int b = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int p1 = min(nc, *pcount);
  const bool live_b = b < p1;
  if (live_b)
    for (int k = threadIdx.x; k < ka; k += blockDim.x)
      rb[k] = C[(int64_t)b * ldc + k];
  __syncthreads();
  for (int a = wave; a < nc; a += blockDim.x / kWave) {
    double v = 0.0;
    if (live_b && a < p1) {
      double s = 0.0;
      const double* ca = C + (int64_t)a * ldc;
      for (int k = lane; k < ka; k += kWave) s += ca[k] * rb[k];
      for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      v = C[(int64_t)hi * ldc + ka + lo] - s;
    }
    if (lane == 0) G2[(int64_t)b * ldg + a] = v;
  }
}

// x(r) += scale * sum_j Q(r, j) y(j), j < k (float64 accumulation, columns
// summed in order).  A wavefront takes 128 rows: lane l reads rows 2l and
// 2l + 1 of its half's 64-row panel as one 2-vector per column, and eight
// columns of loads are issued before their products (a read stream of
// k + 1 columns; one lane-row per thread held the kernel to ~4.9 TB/s).
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_update(
    QView<const T> Q, const double* __restrict__ y, int k,
    const double* __restrict__ sdev, double* __restrict__ x, int64_t n) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  __shared__ double ys[1024];
  const double sc = sdev ? sdev[0] : 1.0;
  const int64_t cs = Q.cstride;
  const int lane = threadIdx.x % kWave;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / kWave) +
                        threadIdx.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int base = 0; base < k; base += 1024) {
    const int kk = min(1024, k - base);
    __syncthreads();
    for (int j = threadIdx.x; j < kk; j += blockDim.x) ys[j] = y[base + j];
    __syncthreads();
    for (int64_t wv = wave0; wv * 128 < n; wv += nwaves) {
      const int64_t r0 = wv * 128 + 2 * lane;  // r0 and r0 + 1: one panel
      if (r0 >= n) continue;
      const T* q = Q.base + Q.row_off(r0) + (int64_t)base * cs;
      double a0 = 0.0, a1 = 0.0;
      int j = 0;
      for (; j + 8 <= kk; j += 8) {
        T2 v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          v[t] = *reinterpret_cast<const T2*>(q + (int64_t)(j + t) * cs);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          a0 += (double)v[t][0] * ys[j + t];
          a1 += (double)v[t][1] * ys[j + t];
        }
      }
      for (; j < kk; ++j) {
        const T2 v = *reinterpret_cast<const T2*>(q + (int64_t)j * cs);
        a0 += (double)v[0] * ys[j];
        a1 += (double)v[1] * ys[j];
      }
      x[r0] += sc * a0;
      if (r0 + 1 < n) x[r0 + 1] += sc * a1;
    }
  }
}

// ------------------------------------------------------------- s = 1
// Column-wise kernels for one-column blocks (the Ritz pre-phase is a run
// of them): MFMA tiles would waste 15 of their 16 columns, so these use
// one row per lane.  Rows are taken in 64-row panels (one per wavefront
// and step), so every column access of a wavefront is one contiguous
// 64-element run.  Sums over rows are per-lane, then a fixed-order
// shuffle tree, then a fixed-order sum over the four wavefronts, then a
// fixed-order sum over workgroups (k_reduce_chunks): deterministic.

// part[chunk][c] = sum over the chunk's rows of Q(r, c) v(r), c < ma, for
// the CT-column tile ct of the grid, v = Q(:, vcol); with *pmask == 0 the
// sums are zero.
template <typename T, int CT>
__global__ __launch_bounds__(kBlock) void k_col_dots(
    QView<const T> Q, int ma, int vcol, const int* __restrict__ pmask,
    int64_t npanels, int ctiles, int chunks, double* __restrict__ part) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int id = blockIdx.x;
  const int xcd = id % 8, slot = id / 8;
  const int ct = slot % ctiles;
  const int chunk = (slot / ctiles) * 8 + xcd;
  const int64_t p0 = npanels * chunk / chunks;
  const int64_t p1 = npanels * (chunk + 1) / chunks;
  const bool live = pmask == nullptr || *pmask > 0;
  const int c0 = ct * CT;
  T acc[CT];
#pragma unroll
  for (int j = 0; j < CT; ++j) acc[j] = (T)0;
  if (live) {
    int64_t oc[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j)
      oc[j] = (int64_t)(c0 + j < ma ? c0 + j : 0) * Q.cstride;
    // narrow tiles: two panels per iteration, all their loads issued
    // together (wide tiles keep one: the registers would cost occupancy)
    constexpr int NWV = kBlock / kWave;
    int64_t pp = p0 + wave;
    if (CT <= 4)
    for (; pp + NWV < p1; pp += 2 * NWV) {
      const T* ra = Q.base + Q.row_off(pp * kPanel) + lane;
      const T* rc = Q.base + Q.row_off((pp + NWV) * kPanel) + lane;
      const T va = ra[(int64_t)vcol * Q.cstride];
      const T vc = rc[(int64_t)vcol * Q.cstride];
      T qa[CT], qc[CT];
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        qa[j] = ra[oc[j]];
        qc[j] = rc[oc[j]];
      }
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[j] += qa[j] * va + qc[j] * vc;
    }
    for (; pp < p1; pp += NWV) {
      const T* rb = Q.base + Q.row_off(pp * kPanel) + lane;
      const T v = rb[(int64_t)vcol * Q.cstride];
      T q[CT];
#pragma unroll
      for (int j = 0; j < CT; ++j) q[j] = rb[oc[j]];
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[j] += q[j] * v;
    }
  }
  __shared__ double red[kBlock / kWave][CT];
#pragma unroll
  for (int j = 0; j < CT; ++j) {
    double t = (double)acc[j];
    for (int off = kWave / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) red[wave][j] = t;
  }
  __syncthreads();
  if (threadIdx.x < CT && c0 + (int)threadIdx.x < ma) {
    const int j = threadIdx.x;
    double t = red[0][j];
    for (int w = 1; w < kBlock / kWave; ++w) t += red[w][j];
    part[(int64_t)chunk * ma + c0 + j] = t;
  }
}

// v = Q(:, vcol) -= Q(:, 0:ma) w (w float64, rounded to T like the MFMA
// update stages it), after v *= *vscale when vscale is given (a previous
// normalisation applied on the way), and part[chunk] = sum of the new
// v(r)^2 over the chunk's rows.  With *pmask == 0 nothing changes and the
// sums are zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_col_update(
    QView<T> Q, int ma, int vcol, const double* __restrict__ w,
    const double* __restrict__ vscale, const int* __restrict__ pmask,
    int64_t npanels, int chunks, double* __restrict__ part) {
  extern __shared__ char smem_raw[];
  T* ws = reinterpret_cast<T*>(smem_raw);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int id = blockIdx.x;
  const int chunk = id;
  const int64_t p0 = npanels * chunk / chunks;
  const int64_t p1 = npanels * (chunk + 1) / chunks;
  const bool live = pmask == nullptr || *pmask > 0;
  for (int j = threadIdx.x; j < ma; j += kBlock) ws[j] = (T)w[j];
  __syncthreads();
  const T sc = (live && vscale) ? (T)vscale[0] : (T)1;
  double ss = 0.0;
  if (live) {
    for (int64_t pp = p0 + wave; pp < p1; pp += kBlock / kWave) {
      T* rb = Q.base + Q.row_off(pp * kPanel) + lane;
      T v = rb[(int64_t)vcol * Q.cstride];
      if (vscale) v = v * sc;
      int j = 0;
      for (; j + 8 <= ma; j += 8) {
        T q[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) q[t] = rb[(int64_t)(j + t) * Q.cstride];
#pragma unroll
        for (int t = 0; t < 8; ++t) v -= q[t] * ws[j + t];
      }
      for (; j < ma; ++j) v -= rb[(int64_t)j * Q.cstride] * ws[j];
      rb[(int64_t)vcol * Q.cstride] = v;
      ss += (double)v * (double)v;
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  __shared__ double red1[kBlock / kWave];
  if (lane == 0) red1[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red1[0];
    for (int k = 1; k < kBlock / kWave; ++k) t += red1[k];
    part[chunk] = t;
  }
}

// The first CGS pass of a one-column block with the second pass's
// projection in the same sweep: v' = Q(:, vcol) -= Q(:, 0:ma) w (w float64,
// rounded to T and subtracted in the same column order as in
// k_col_update), and per chunk
// part[chunk][0:ma] = sum over the chunk's rows of Q(r, c) v'(r) and
// part[chunk][ma] = sum of v'(r)^2.  The MA <= 32 columns of a row stay in
// registers between the update and the dot products, so Q(:, 0:ma) is read
// once for both; absent columns (ma < MA) load column 0 and get weight 0,
// their dot products are not stored.
template <typename T, int MA>
__global__ __launch_bounds__(kBlock) void k_col_update_dots(
    QView<T> Q, int ma, int vcol, const double* __restrict__ w,
    int64_t npanels, int chunks, double* __restrict__ part) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int chunk = blockIdx.x;
  const int64_t p0 = npanels * chunk / chunks;
  const int64_t p1 = npanels * (chunk + 1) / chunks;
  T wt[MA];
  int64_t oc[MA];
#pragma unroll
  for (int j = 0; j < MA; ++j) {
    wt[j] = j < ma ? (T)w[j] : (T)0;
    oc[j] = (int64_t)(j < ma ? j : 0) * Q.cstride;
  }
  T acc[MA];
#pragma unroll
  for (int j = 0; j < MA; ++j) acc[j] = (T)0;
  double ss = 0.0;
  for (int64_t pp = p0 + wave; pp < p1; pp += kBlock / kWave) {
    T* rb = Q.base + Q.row_off(pp * kPanel) + lane;
    T v = rb[(int64_t)vcol * Q.cstride];
    T q[MA];
#pragma unroll
    for (int j = 0; j < MA; ++j) q[j] = rb[oc[j]];
#pragma unroll
    for (int j = 0; j < MA; ++j) v -= q[j] * wt[j];
    rb[(int64_t)vcol * Q.cstride] = v;
    ss += (double)v * (double)v;
#pragma unroll
    for (int j = 0; j < MA; ++j) acc[j] += q[j] * v;
  }
  __shared__ double red[kBlock / kWave][MA + 1];
#pragma unroll
  for (int j = 0; j <= MA; ++j) {
    double t = j < MA ? (double)acc[j] : ss;
    for (int off = kWave / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) red[wave][j] = t;
  }
  __syncthreads();
  const int e = threadIdx.x;
  if (e <= ma) {
    const int src = e < ma ? e : MA;
    double t = red[0][src];
    for (int k = 1; k < kBlock / kWave; ++k) t += red[k][src];
    part[(int64_t)chunk * (ma + 1) + e] = t;
  }
}

// The same pass for 32 < ma <= 256 prior columns: the K = blockDim / 64
// wavefronts of a workgroup walk the chunk's panels together, wavefront w
// holding columns [32 w, 32 w + 32) of the panel's rows in registers.
// Each forms its share of Q w for its rows; the shares meet in LDS and
// every wavefront subtracts them from v in the same order, so all of them
// hold the same v'; wavefront 0 stores it and keeps the square sum, and
// each wavefront accumulates the dot products of its own columns.  Two LDS
// slots alternate between panels, so one barrier per panel suffices.
constexpr int kColWave = 32;      // columns per wavefront
constexpr int kColWideMax = 256;  // 8 wavefronts
template <typename T>
__global__ __launch_bounds__(kColWideMax / kColWave * kWave) void
k_col_update_dots_wide(QView<T> Q, int ma, int vcol,
                       const double* __restrict__ w, int64_t npanels,
                       int chunks, double* __restrict__ part) {
  constexpr int CW = kColWave;
  constexpr int KMAX = kColWideMax / kColWave;
  __shared__ T share[2][KMAX][kWave];
  __shared__ double red[KMAX][CW + 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nwv = blockDim.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int chunk = blockIdx.x;
  const int64_t p0 = npanels * chunk / chunks;
  const int64_t p1 = npanels * (chunk + 1) / chunks;
  const int c0 = wave * CW;
  T wt[CW];
  int64_t oc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) {
    const bool in = c0 + j < ma;
    wt[j] = in ? (T)w[c0 + j] : (T)0;
    oc[j] = (int64_t)(in ? c0 + j : 0) * Q.cstride;
  }
  T acc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) acc[j] = (T)0;
  double ss = 0.0;
  int slot = 0;
  for (int64_t pp = p0; pp < p1; ++pp, slot ^= 1) {
    T* rb = Q.base + Q.row_off(pp * kPanel) + lane;
    const T v = rb[(int64_t)vcol * Q.cstride];
    T q[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) q[j] = rb[oc[j]];
    T y = (T)0;
#pragma unroll
    for (int j = 0; j < CW; ++j) y += q[j] * wt[j];
    share[slot][wave][lane] = y;
    __syncthreads();
    T vn = v;
    for (int k = 0; k < nwv; ++k) vn -= share[slot][k][lane];
    if (wave == 0) {
      rb[(int64_t)vcol * Q.cstride] = vn;
      ss += (double)vn * (double)vn;
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[j] += q[j] * vn;
  }
#pragma unroll
  for (int j = 0; j <= CW; ++j) {
    double t = j < CW ? (double)acc[j] : ss;
    for (int off = kWave / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) red[wave][j] = t;
  }
  __syncthreads();
  // dots of column c from its wavefront's row, the square sum from wave 0
  for (int e = threadIdx.x; e <= ma; e += blockDim.x) {
    const double t = e < ma ? red[e / CW][e % CW] : red[0][CW];
    part[(int64_t)chunk * (ma + 1) + e] = t;
  }
}

// Fixed-order sum over the chunks of ne = ndots + norm partials (ndots dot
// products, then with norm the square sum g), kRedOut outputs at a time as
// in k_reduce_chunks.  live = (pmask == NULL or *pmask > 0).
// - With norm: the partial Cholesky of the 1 x 1 Gram g (Alg. 3 with
//   s = 1: the pivot alone decides, one column's condition estimate is 1):
//   *p_out = 1, R[0] = sqrt(g), Rinv[0] = 1 / R[0] when live and g > 0 is
//   finite, else *p_out = 0 and R, Rinv untouched.
// - dots_out[0:ndots] = the dots times *dscale (when given), zero when not
//   live.
// - With norm_scales (needs norm and ndots <= 256): the dots are scaled by
//   the 1 / R[0] just computed instead, and are zero when *p_out = 0 (the
//   second CGS projection of the normalised vector, from the sums of the
//   unnormalised one).
__global__ __launch_bounds__(kRedThreads) void k_col_finish(
    const double* __restrict__ part, int64_t nchunks, int ndots, int norm,
    const int* __restrict__ pmask, const double* __restrict__ dscale,
    double* __restrict__ dots_out, double* __restrict__ R,
    double* __restrict__ Rinv, int* p_out, int norm_scales) {
  __shared__ double red[kRedThreads];
  __shared__ double sums[kColWideMax];
  __shared__ double gsum, gscale;
  __shared__ int gok;
  const int o = threadIdx.x % kRedOut, g = threadIdx.x / kRedOut;
  const int ne = ndots + norm;
  const bool live = pmask == nullptr || *pmask > 0;
  const double sc = (live && dscale) ? dscale[0] : 1.0;
  for (int e0 = 0; e0 < ne; e0 += kRedOut) {
    const int e = e0 + o;
    red[threadIdx.x] = e < ne ? chunk_sum(part, nchunks, ne, e, g) : 0.0;
    group_tree(red);
    if (g == 0 && e < ne) {
      const double t = red[o];
      if (e < ndots) {
        if (norm_scales)
          sums[e] = t;
        else if (dots_out)
          dots_out[e] = live ? t * sc : 0.0;
      } else {
        gsum = t;
      }
    }
    __syncthreads();
  }
  if (norm && threadIdx.x == 0) {
    const double g = gsum;
    const bool ok = live && g > 0.0 && isfinite(g);
    if (ok) {
      const double r = sqrt(g);
      R[0] = r;
      Rinv[0] = 1.0 / r;
    }
    *p_out = ok ? 1 : 0;
    gok = ok ? 1 : 0;
    gscale = ok ? 1.0 / sqrt(g) : 0.0;
  }
  if (norm_scales) {
    __syncthreads();
    for (int e = threadIdx.x; e < ndots; e += blockDim.x)
      dots_out[e] = gok ? sums[e] * gscale : 0.0;
  }
}

// v = Q(:, vcol) *= (T) *z when *pmask > 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_col_scale(
    QView<T> Q, int vcol, const double* __restrict__ z,
    const int* __restrict__ pmask, int64_t nrows) {
  if (pmask != nullptr && *pmask <= 0) return;
  const T zz = (T)z[0];
  for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * kBlock) {
    T* p = Q.at(r, vcol);
    *p = *p * zz;
  }
}

// ------------------------------------------------------------- dispatch
// About two workgroups per CU (256 CUs): one full wave of workgroups, few
// enough partials that their reduction stays cheap.
constexpr int kTargetGroups = 512;
constexpr int kNumCUs = 256;  // MI355X compute units

int pick_chunks(int target_groups, int ntiles, int64_t nbatches,
                int64_t per_chunk, const Partials& P) {
  int64_t target = (target_groups + ntiles - 1) / ntiles;
  int64_t maxc = nbatches / 4;  // at least one batch per wavefront
  if (target > maxc) target = maxc;
  int64_t capc = per_chunk > 0 ? P.cap / per_chunk : target;
  if (target > capc) target = capc;
  target = target / 8 * 8;
  if (target < 8) target = 8;
  if (target * per_chunk > P.cap)
    throw Error{SGM_EINVAL, "partial-sum scratch too small for this block"};
  return (int)target;
}

template <typename T, int MT, int NT, int WT, bool SYM = false>
void launch_gemm_tn(QView<const T> Q, int a0, int ma, int b0, int nb,
                    const int* ncount, int64_t nbatches, int wtiles_n,
                    int n_wtiles, int ngroups, int chunks, double* part,
                    hipStream_t st) {
  hipLaunchKernelGGL((k_gemm_tn<T, MT, NT, WT, SYM>), dim3(chunks * ngroups),
                     dim3(kBlock), 0, st, Q, a0, ma, b0, nb, ncount, nbatches,
                     wtiles_n, n_wtiles, ngroups, chunks, part);
  SGM_CHECK_LAUNCH();
}

}  // namespace

// Shape choice (from a sweep over the block shapes of the solver on
// 2M-row panels): NT column tiles per wave tile (1, 2 or 4); MT row tiles
// up to MT * NT = 8 (float64) or 16 (float32); WT = 2 wave tiles per
// workgroup when there are at least two, else one wave tile with the
// wavefronts on four row phases (splitting the output further makes the
// wavefronts re-read the shared B columns and costs more than it gains).
// The grid holds about 256 workgroups for the largest wave tiles and up to
// 1024 for the smallest, so the bytes in flight stay near the same level.
template <typename T>
void gemm_tn(QView<const T> Q, int a0, int ma, int b0, int nb,
             const int* ncount, int64_t nrows, double* C, int ldc,
             Partials& P, hipStream_t st) {
  if (ma <= 0 || nb <= 0) return;
  const int mt_all = (ma + 15) / 16, nt_all = (nb + 15) / 16;
  const int NT = nt_all <= 1 ? 1 : (nt_all <= 2 ? 2 : 4);
  const int max_tiles = sizeof(T) == 8 ? 8 : 16;
  int MT = 1;
  while (MT < mt_all && MT < 8 && 2 * MT * NT <= max_tiles) MT *= 2;
  const int wtiles_n = (nt_all + NT - 1) / NT;
  const int wtiles_m = (mt_all + MT - 1) / MT;
  const int n_wtiles = wtiles_m * wtiles_n;
  const int WT = n_wtiles >= 2 ? 2 : 1;
  const int ngroups = (n_wtiles + WT - 1) / WT;
  const int64_t nbatches = (nrows + 15) / 16;
  int64_t groups = (int64_t)256 * 64 / ((int64_t)MT * NT * sizeof(T));
  groups = groups < 256 ? 256 : (groups > 1024 ? 1024 : groups);
  const int chunks =
      pick_chunks((int)groups, ngroups, nbatches, (int64_t)ma * nb, P);
  if (mt_all > kWM && mt_all <= kRM && nt_all > 6 &&
      !(a0 == b0 && ma == nb)) {
    // 145 to 208 rows, more than 96 columns: all rows per workgroup
    // (measured at 201 x 200 over 16.8M rows, float64: see the kernel)
    const int nblk = (nt_all + kRN - 1) / kRN;
    const int chunks_t =
        pick_chunks(2 * kNumCUs, nblk, nbatches, (int64_t)ma * nb, P);
    const size_t lds = (size_t)2 * kRCols * kWStride * sizeof(T);
    hipLaunchKernelGGL(k_gemm_tn_tall<T>, dim3(chunks_t * nblk),
                       dim3(kRBlock), lds, st, Q, a0, ma, b0, nb, ncount,
                       nbatches, nblk, chunks_t, P.buf);
    SGM_CHECK_LAUNCH();
    launch_reduce(P.buf, chunks_t, ma, nb, C, ldc, 0, st);
    return;
  }
  if (mt_all > 4 && nt_all > 6 && !(a0 == b0 && ma == nb)) {
    // more than 64 rows and 96 columns, not a Gram matrix: the LDS-shared
    // kernel, whose 144 x 128 blocks are then mostly full (measured in the
    // 192^3 solve at 129 x 128: 4.6 against 6.6 ms in float64, 2.4 against
    // 3.6 ms in float32; a one-row product would waste 8 of its 9 row
    // tiles)
    const int nbm = (ma + 16 * kWM - 1) / (16 * kWM);
    const int nbn = (nb + 16 * kWN - 1) / (16 * kWN);
    const int nblk = nbm * nbn;
    const int chunks_w =
        pick_chunks(2 * kNumCUs, nblk, nbatches, (int64_t)ma * nb, P);
    const size_t lds = (size_t)2 * kWCols * kWStride * sizeof(T);
    hipLaunchKernelGGL(k_gemm_tn_wide<T>, dim3(chunks_w * nblk),
                       dim3(kWBlock), lds, st, Q, a0, ma, b0, nb, ncount,
                       nbatches, nbn, nblk, chunks_w, P.buf);
    SGM_CHECK_LAUNCH();
    launch_reduce(P.buf, chunks_w, ma, nb, C, ldc, 0, st);
    return;
  }
  // A Gram matrix of 129 to 256 columns: every 32- or 16-row batch of its
  // columns in LDS once per workgroup, the tiles on and above the diagonal formed
  // from there (the kernels below fetch each operand per wavefront).
  // Measured in float64: 200 columns over 16.8M rows 14.7 against 33.6 ms;
  // at 128 columns over 7.1M rows the kernel below is faster (4.2 against
  // 4.7 ms), so it keeps those.
  if (a0 == b0 && ma == nb && nb > 128 && nb <= kGMaxCols) {
    // at most 7 tiles per wavefront up to 224 columns (105 tiles): 32-row
    // batches; 9 up to 256: 16-row batches (the rows past nrows up to the
    // 64-row panel boundary are zero)
    const bool seven = nt_all * (nt_all + 1) / 2 <= 7 * kGWaves;
    const int rows = seven ? 32 : 16;
    const int64_t gbatches = (nrows + rows - 1) / rows;
    const int chunks_g =
        pick_chunks(2 * kNumCUs, 1, gbatches, (int64_t)nb * nb, P);
    const size_t lds = (size_t)2 * nt_all * 16 * (rows + 1) * sizeof(T);
    if (seven)
      hipLaunchKernelGGL((k_gram_wide<T, 7, 32>), dim3(chunks_g),
                         dim3(kGBlock), lds, st, Q, b0, nb, ncount, gbatches,
                         chunks_g, P.buf);
    else
      hipLaunchKernelGGL((k_gram_wide<T, kGTiles, 16>), dim3(chunks_g),
                         dim3(kGBlock), lds, st, Q, b0, nb, ncount, gbatches,
                         chunks_g, P.buf);
    SGM_CHECK_LAUNCH();
    launch_reduce(P.buf, chunks_g, nb, nb, C, ldc, 1, st);
    return;
  }
  // A float64 Gram matrix wider than 64 columns: 64 x 64 wave tiles, one
  // per wavefront, on and above the diagonal only.  (Measured at 128
  // columns over 7M rows: 4.1 ms against 4.5 ms for the full product in
  // 32 x 64 tiles.  The kernel is bound by fetching its operands, not by
  // the matrix cores, so the larger tiles gain more than the skipped
  // tiles; in float32 the full product measured faster.)
  if (sizeof(T) == 8 && a0 == b0 && ma == nb && nt_all > 4) {
    // 2048 workgroups, of which those below the diagonal idle at once
    // (at 200 columns: 34 against 38 ms with 256)
    const int wn = (nt_all + 3) / 4, wm = (mt_all + 3) / 4;
    const int chunks_s =
        pick_chunks(8 * kNumCUs, wm * wn, nbatches, (int64_t)ma * nb, P);
    launch_gemm_tn<T, 4, 4, 1, true>(Q, a0, ma, b0, nb, ncount, nbatches, wn,
                                     wm * wn, wm * wn, chunks_s, P.buf, st);
    launch_reduce(P.buf, chunks_s, ma, nb, C, ldc, 1, st);
    return;
  }
#define SGM_GT(mt, nt, wt)                                                  \
  if (MT == mt && NT == nt && WT == wt) {                                   \
    launch_gemm_tn<T, mt, nt, wt>(Q, a0, ma, b0, nb, ncount, nbatches,      \
                                  wtiles_n, n_wtiles, ngroups, chunks,      \
                                  P.buf, st);                               \
  } else
  SGM_GT(1, 1, 1) SGM_GT(2, 1, 1) SGM_GT(4, 1, 1) SGM_GT(8, 1, 1)
  SGM_GT(1, 1, 2) SGM_GT(2, 1, 2) SGM_GT(4, 1, 2) SGM_GT(8, 1, 2)
  SGM_GT(1, 2, 1) SGM_GT(2, 2, 1) SGM_GT(4, 2, 1) SGM_GT(8, 2, 1)
  SGM_GT(1, 2, 2) SGM_GT(2, 2, 2) SGM_GT(4, 2, 2) SGM_GT(8, 2, 2)
  SGM_GT(1, 4, 1) SGM_GT(2, 4, 1) SGM_GT(4, 4, 1)
  SGM_GT(1, 4, 2) SGM_GT(2, 4, 2) SGM_GT(4, 4, 2)
  { throw Error{SGM_EINVAL, "gemm_tn: no kernel for this shape"}; }
#undef SGM_GT
  launch_reduce(P.buf, chunks, ma, nb, C, ldc, 0, st);
}

namespace {

constexpr int kLdsBudget = 64 * 1024;
// LDS of one workgroup for the staged M of blocks wider than 64 columns:
// most of gfx950's 160 KiB, so M stays whole for i + s up to about 150
// (float64) or 300 (float32) at s = 128.
constexpr int kWideLdsBudget = 152 * 1024;

// Largest LDS of one workgroup on gfx950 (bytes).
constexpr int kMaxLds = 160 * 1024;

template <typename T, int NT, int MT, int MODE, bool GRAM, int BLOCK>
void launch_update_b(QView<T> Q, int a0, int ka, int b0, int nc,
                     const double* M, int ldm, const int* ncount,
                     int64_t nrows, double* G, int ldg, Partials& P,
                     hipStream_t st, int lds_budget, int64_t target_groups) {
  const int W16 = NT * 16;
  const int ka4 = (ka + 3) & ~3;
  int kc = lds_budget / (W16 * (int)sizeof(T));
  kc &= ~3;
  if constexpr (MODE == MODE_TRSM && !GRAM && NT > 4 && sizeof(T) == 8) {
    // a float64 triangular factor that does not fit whole: packed, when
    // that fits (float32 factors fit whole up to 197 columns)
    // (plus room for the reads past the triangle's last row: W16 + 64)
    const size_t packed = ((size_t)nc * (nc + 1) / 2 + W16 + 64) * sizeof(T);
    if (kc < ka4 && packed <= (size_t)kMaxLds) {
      const int64_t rows_per_block = 16 * MT * (BLOCK / kWave);
      const int64_t nblocks = ceil_div(nrows, rows_per_block);
      int64_t grid = nblocks < target_groups ? nblocks : target_groups;
      if (grid < 1) grid = 1;
      hipLaunchKernelGGL((k_update<T, NT, MT, MODE, false, BLOCK, true>),
                         dim3((unsigned)grid), dim3(BLOCK), packed, st, Q, a0,
                         ka, b0, nc, M, ldm, ncount, nrows, ka4,
                         (double*)nullptr);
      SGM_CHECK_LAUNCH();
      return;
    }
  }
  if (kc > ka4) kc = ka4 < 4 ? 4 : ka4;
  size_t lds = (size_t)kc * W16 * sizeof(T);
  if (GRAM) {
    const size_t red = (size_t)(NT * (NT + 1) / 2) * 4 * kWave * sizeof(double);
    if (red > lds) lds = red;
  }
  const int64_t rows_per_block = 16 * MT * (BLOCK / kWave);
  const int64_t nblocks = ceil_div(nrows, rows_per_block);
  int64_t grid = nblocks < target_groups ? nblocks : target_groups;
  if (grid < 1) grid = 1;
  if (GRAM && grid * nc * nc > P.cap) {
    grid = P.cap / ((int64_t)nc * nc);
    if (grid < 1) throw Error{SGM_EINVAL, "partial scratch too small"};
  }
  hipLaunchKernelGGL((k_update<T, NT, MT, MODE, GRAM, BLOCK>),
                     dim3((unsigned)grid), dim3(BLOCK), lds, st, Q, a0, ka,
                     b0, nc, M, ldm, ncount, nrows, kc,
                     GRAM ? P.buf : (double*)nullptr);
  SGM_CHECK_LAUNCH();
  if (GRAM) launch_reduce(P.buf, grid, nc, nc, G, ldg, 1, st);
}

// Blocks up to 64 columns: 256-thread workgroups, a 64 KiB chunk of M.
// Wider blocks: one workgroup per CU holding (most of) M in LDS, with 1024
// threads while the kernel fits four wavefronts per SIMD (at most 128
// registers each: up to 72 accumulator registers), else 512.
template <typename T, int NT, int MT, int MODE, bool GRAM>
void launch_update(QView<T> Q, int a0, int ka, int b0, int nc,
                   const double* M, int ldm, const int* ncount, int64_t nrows,
                   double* G, int ldg, Partials& P, hipStream_t st,
                   int target_groups = kTargetGroups) {
  if constexpr (NT <= 4 || GRAM) {
    launch_update_b<T, NT, MT, MODE, GRAM, kBlock>(
        Q, a0, ka, b0, nc, M, ldm, ncount, nrows, G, ldg, P, st, kLdsBudget,
        target_groups);
  } else {
    constexpr int acc_regs = NT * MT * 4 * (int)sizeof(T) / 4;
    constexpr int B = acc_regs <= 72 ? 1024 : 512;
    launch_update_b<T, NT, MT, MODE, GRAM, B>(
        Q, a0, ka, b0, nc, M, ldm, ncount, nrows, G, ldg, P, st,
        kWideLdsBudget, kNumCUs);
  }
}

}  // namespace

// One column group of a wide update: 16 nt columns from column c0 of the
// block (rows c0 .. of M), on the wide path (1,024 threads, the group's
// slice of M staged whole in LDS).
template <typename T, int NT>
void launch_update_group(QView<T> Q, int a0, int ka, int b0, int c0, int ncg,
                         const double* M, int ldm, const int* ncount,
                         int64_t nrows, hipStream_t st) {
  const int W16 = NT * 16;
  const int ka4 = (ka + 3) & ~3;
  const size_t lds = (size_t)ka4 * W16 * sizeof(T);
  const int64_t rows_per_block = 16 * (1024 / kWave);
  const int64_t nblocks = ceil_div(nrows, rows_per_block);
  int64_t grid = nblocks < kNumCUs ? nblocks : kNumCUs;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_update<T, NT, 1, MODE_UPDATE, false, 1024>),
                     dim3((unsigned)grid), dim3(1024), lds, st, Q, a0, ka,
                     b0 + c0, ncg, M + (int64_t)c0 * ldm, ldm, ncount, nrows,
                     ka4, (double*)nullptr, c0);
  SGM_CHECK_LAUNCH();
}

// Column groups of at most 80 columns when the whole coefficient matrix M
// (ka x nc) does not fit the wide kernel's LDS: each group's slice of M
// then stays in LDS for the whole pass instead of being re-staged in
// chunks for every row block.  The prior columns are read once per group.
// Measured in float64 at ka = 201, nc = 200 over 16.8M rows (M 321 KB).
template <typename T>
bool update_in_groups(QView<T> Q, int a0, int ka, int b0, int nc,
                      const double* M, int ldm, const int* ncount,
                      int64_t nrows, hipStream_t st) {
  const int ka4 = (ka + 3) & ~3;
  const size_t whole = (size_t)ka4 * ((nc + 15) / 16) * 16 * sizeof(T);
  if (whole <= (size_t)kWideLdsBudget) return false;
  int wcols = (int)(kWideLdsBudget / ((size_t)ka4 * sizeof(T))) / 16 * 16;
  if (wcols > 80) wcols = 80;
  if (wcols < 16) return false;
  for (int c0 = 0; c0 < nc; c0 += wcols) {
    const int ncg = nc - c0 < wcols ? nc - c0 : wcols;
    switch ((ncg + 15) / 16) {
      case 1: launch_update_group<T, 1>(Q, a0, ka, b0, c0, ncg, M, ldm, ncount, nrows, st); break;
      case 2: launch_update_group<T, 2>(Q, a0, ka, b0, c0, ncg, M, ldm, ncount, nrows, st); break;
      case 3: launch_update_group<T, 3>(Q, a0, ka, b0, c0, ncg, M, ldm, ncount, nrows, st); break;
      case 4: launch_update_group<T, 4>(Q, a0, ka, b0, c0, ncg, M, ldm, ncount, nrows, st); break;
      default: launch_update_group<T, 5>(Q, a0, ka, b0, c0, ncg, M, ldm, ncount, nrows, st); break;
    }
  }
  return true;
}

template <typename T>
void update_gram(QView<T> Q, int a0, int ka, int b0, int nc, const double* M,
                 int ldm, const int* ncount, int64_t nrows, double* G,
                 int ldg, Partials& P, hipStream_t st) {
  if (nc <= 0) return;
  const int nt = (nc + 15) / 16;
  const bool fuse = G != nullptr && nt <= 4;
  if (!fuse && nt > 4 &&
      update_in_groups<T>(Q, a0, ka, b0, nc, M, ldm, ncount, nrows, st)) {
    if (G != nullptr)
      gemm_tn<T>(Q.template as<const T>(), b0, nc, b0, nc, ncount, nrows, G,
                 ldg, P, st);
    return;
  }
#define SGM_UP(NTv, MTv)                                                      \
  if (nt == NTv) {                                                            \
    if (fuse)                                                                 \
      launch_update<T, NTv, MTv, MODE_UPDATE, (NTv <= 4)>(                    \
          Q, a0, ka, b0, nc, M, ldm, ncount, nrows, G, ldg, P, st);           \
    else                                                                      \
      launch_update<T, NTv, MTv, MODE_UPDATE, false>(                         \
          Q, a0, ka, b0, nc, M, ldm, ncount, nrows, nullptr, 0, P, st);       \
  } else
  SGM_UP(1, 4) SGM_UP(2, 4) SGM_UP(3, 2) SGM_UP(4, 2) SGM_UP(5, 1)
  SGM_UP(6, 1) SGM_UP(7, 1) SGM_UP(8, 1) SGM_UP(9, 1) SGM_UP(10, 1)
  SGM_UP(11, 1) SGM_UP(12, 1) SGM_UP(13, 1) SGM_UP(14, 1) SGM_UP(15, 1)
  SGM_UP(16, 1)
  { throw Error{SGM_EINVAL, "update: block wider than 256 columns"}; }
#undef SGM_UP
  if (G != nullptr && !fuse)
    gemm_tn<T>(Q.template as<const T>(), b0, nc, b0, nc, ncount, nrows, G,
               ldg, P, st);
}

template <typename T>
void trsm_inv(QView<T> Q, int b0, int s, const double* Rinv, int ldr,
              const int* pcount, int64_t nrows, hipStream_t st) {
  if (s <= 0) return;
  Partials none;
  const int nt = (s + 15) / 16;
  if (sizeof(T) == 4 && nt <= 2) {
    // float32, narrow: 32 rows per wavefront and more workgroups keep more
    // bytes in flight (measured: 3.8 -> 4.6 TB/s at 32 columns)
    if (nt == 1)
      launch_update<T, 1, 2, MODE_TRSM, false>(Q, 0, s, b0, s, Rinv, ldr,
                                               pcount, nrows, nullptr, 0,
                                               none, st, 1024);
    else
      launch_update<T, 2, 2, MODE_TRSM, false>(Q, 0, s, b0, s, Rinv, ldr,
                                               pcount, nrows, nullptr, 0,
                                               none, st, 1024);
    return;
  }
  if (sizeof(T) == 8 && nt == 13) {
    // 193 to 208 float64 columns, factor packed in LDS: two 16-row tiles
    // per wavefront and one wavefront per SIMD (256 threads: 512 registers
    // a lane), so each read of the factor feeds two MFMAs
    launch_update_b<T, 13, 2, MODE_TRSM, false, 256>(
        Q, 0, s, b0, s, Rinv, ldr, pcount, nrows, nullptr, 0, none, st,
        kWideLdsBudget, kNumCUs);
    return;
  }
#define SGM_TR(NTv, MTv)                                                      \
  if (nt == NTv) {                                                            \
    launch_update<T, NTv, MTv, MODE_TRSM, false>(                             \
        Q, 0, s, b0, s, Rinv, ldr, pcount, nrows, nullptr, 0, none, st);      \
  } else
  SGM_TR(1, 4) SGM_TR(2, 4) SGM_TR(3, 2) SGM_TR(4, 2) SGM_TR(5, 1)
  SGM_TR(6, 1) SGM_TR(7, 1) SGM_TR(8, 1) SGM_TR(9, 1) SGM_TR(10, 1)
  SGM_TR(11, 1) SGM_TR(12, 1) SGM_TR(13, 1) SGM_TR(14, 1) SGM_TR(15, 1)
  SGM_TR(16, 1)
  { throw Error{SGM_EINVAL, "trsm: block wider than 256 columns"}; }
#undef SGM_TR
}

template <typename T>
bool trsm_inv_gram(QView<T> Q, int b0, int s, const double* Rinv, int ldr,
                   const int* pcount, int64_t nrows, double* G, int ldg,
                   Partials& P, hipStream_t st) {
  const int nt = (s + 15) / 16;
  if (s <= 0 || nt > 4) return false;
  if (sizeof(T) == 4 && nt <= 2) {
    if (nt == 1)
      launch_update<T, 1, 2, MODE_TRSM, true>(Q, 0, s, b0, s, Rinv, ldr,
                                              pcount, nrows, G, ldg, P, st,
                                              1024);
    else
      launch_update<T, 2, 2, MODE_TRSM, true>(Q, 0, s, b0, s, Rinv, ldr,
                                              pcount, nrows, G, ldg, P, st,
                                              1024);
    return true;
  }
  if (nt == 1)
    launch_update<T, 1, 4, MODE_TRSM, true>(Q, 0, s, b0, s, Rinv, ldr, pcount,
                                            nrows, G, ldg, P, st);
  else if (nt == 2)
    launch_update<T, 2, 4, MODE_TRSM, true>(Q, 0, s, b0, s, Rinv, ldr, pcount,
                                            nrows, G, ldg, P, st);
  else if (nt == 3)
    launch_update<T, 3, 2, MODE_TRSM, true>(Q, 0, s, b0, s, Rinv, ldr, pcount,
                                            nrows, G, ldg, P, st);
  else
    launch_update<T, 4, 2, MODE_TRSM, true>(Q, 0, s, b0, s, Rinv, ldr, pcount,
                                            nrows, G, ldg, P, st);
  return true;
}

template <typename T>
void gemv_update(QView<const T> Q, const double* y, int k,
                 const double* sdev, double* x, int64_t n, hipStream_t st) {
  if (k <= 0) return;
  int64_t grid = ceil_div(n, 4 * 128);  // four 128-row wavefronts per group
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_gemv_update<T>, dim3((unsigned)grid), dim3(256), 0,
                     st, Q, y, k, sdev, x, n);
  SGM_CHECK_LAUNCH();
}

namespace {
template <typename T, int NT, int MQ>
void launch_trsm_proj(QView<T> Q, int ka, int b0, int nc, const double* Zinv,
                      int ldz, const int* pcount, int64_t nrows, double* R2,
                      int ldr, Partials& P, hipStream_t st) {
  constexpr int MT = 4;
  const int64_t rows_per_block = 16 * MT * (kBlock / kWave);
  const int64_t nblocks = ceil_div(nrows, rows_per_block);
  int64_t grid = nblocks < kTargetGroups ? nblocks : kTargetGroups;
  if (grid < 1) grid = 1;
  if (grid * ka * nc > P.cap) grid = P.cap / ((int64_t)ka * nc);
  if (grid < 1) throw Error{SGM_EINVAL, "partial scratch too small"};
  const size_t stage = (size_t)(((nc + 3) & ~3)) * NT * 16 * sizeof(T);
  const size_t red = (size_t)MQ * NT * 4 * kWave * sizeof(double);
  const size_t lds = stage > red ? stage : red;
  hipLaunchKernelGGL((k_trsm_proj<T, NT, MT, MQ>), dim3((unsigned)grid),
                     dim3(kBlock), lds, st, Q, ka, b0, nc, Zinv, ldz, pcount,
                     nrows, P.buf);
  SGM_CHECK_LAUNCH();
  launch_reduce(P.buf, grid, ka, nc, R2, ldr, 0, st);
}
}  // namespace

// Used where it measured faster than the two separate passes: float64
// with at most 64 prior columns (3D Poisson 128^3, 33 x 32 block: 422 ->
// 359 us).  With more columns the projection's accumulators drop the
// kernel to one wavefront per SIMD and the separate passes win; in float32
// the separate passes are as fast or faster.
template <typename T>
bool trsm_proj(QView<T> Q, int ka, int b0, int nc, const double* Zinv,
               int ldz, const int* pcount, int64_t nrows, double* R2, int ldr,
               Partials& P, hipStream_t st) {
  if (sizeof(T) != 8 || ka < 1 || nc < 2 || ka > 64 || nc > 32) return false;
  const int nt = (nc + 15) / 16, mq = (ka + 15) / 16;
#define SGM_TP(NTv, MQv)                                                      \
  if (nt == NTv && mq <= MQv) {                                               \
    launch_trsm_proj<T, NTv, MQv>(Q, ka, b0, nc, Zinv, ldz, pcount, nrows,    \
                                  R2, ldr, P, st);                            \
    return true;                                                              \
  }
  SGM_TP(1, 2) SGM_TP(1, 4)
  SGM_TP(2, 2) SGM_TP(2, 4)
#undef SGM_TP
  return false;
}

// Fused when Zinv fits in LDS beside the staged M (up to 64 columns);
// wider blocks take the plain update and the triangular solve as two
// passes.
template <typename T>
void update_trsm(QView<T> Q, int ka, int b0, int nc, const double* M,
                 int ldm, const double* Zinv, int ldz, const int* pcount,
                 int64_t nrows, hipStream_t st) {
  if (nc <= 0) return;
  const int nt = (nc + 15) / 16;
  if (nt > 4) {
    Partials none;
    update_gram<T>(Q, 0, ka, b0, nc, M, ldm, pcount, nrows, nullptr, 0, none,
                   st);
    trsm_inv<T>(Q, b0, nc, Zinv, ldz, pcount, nrows, st);
    return;
  }
  auto launch = [&](auto nt_c, auto mt_c) {
    constexpr int NTv = decltype(nt_c)::value, MTv = decltype(mt_c)::value;
    constexpr int W16 = NTv * 16;
    const int ka4 = (ka + 3) & ~3;
    int kc = kLdsBudget / (W16 * (int)sizeof(T));
    kc &= ~3;
    if (kc > ka4) kc = ka4 < 4 ? 4 : ka4;
    const size_t lds = (size_t)(W16 * W16 + kc * W16) * sizeof(T);
    const int64_t rows_per_block = 16 * MTv * (kBlock / kWave);
    const int64_t nblocks = ceil_div(nrows, rows_per_block);
    int64_t grid = nblocks < kTargetGroups ? nblocks : kTargetGroups;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_update_trsm<T, NTv, MTv>), dim3((unsigned)grid),
                       dim3(kBlock), lds, st, Q, ka, b0, nc, M, ldm, Zinv,
                       ldz, pcount, nrows, kc);
    SGM_CHECK_LAUNCH();
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  if (nt == 1) launch(I1{}, I4{});
  else if (nt == 2) launch(I2{}, I4{});
  else if (nt == 3) launch(I3{}, I2{});
  else launch(I4{}, I2{});
}

void pyth_gram(const double* C, int ldc, int ka, int nc, const int* pcount,
               double* G2, int ldg, hipStream_t st) {
  if (nc <= 0) return;
  if ((size_t)ka * sizeof(double) > 64 * 1024)
    throw Error{SGM_EINVAL, "pyth_gram: too many prior columns"};
  const size_t lds = sizeof(double) * (size_t)(ka > 0 ? ka : 1);
  hipLaunchKernelGGL(k_pyth_gram, dim3((unsigned)nc), dim3(256), lds, st, C,
                     ldc, ka, nc, pcount, G2, ldg);
  SGM_CHECK_LAUNCH();
}

namespace {
// Row chunks of the column-wise kernels: about 1024 workgroups, at least
// four panels (one per wavefront) each, a multiple of 8 for the XCD
// decode, and within the partial-sum scratch.
int col_chunks(int64_t npanels, int ctiles, int64_t per_chunk,
               const Partials& P) {
  int64_t c = 1024 / ctiles;
  if (c > npanels / 4) c = npanels / 4;
  if (per_chunk > 0 && c > P.cap / per_chunk) c = P.cap / per_chunk;
  c = c / 8 * 8;
  if (c < 8) c = 8;
  if (c * per_chunk > P.cap)
    throw Error{SGM_EINVAL, "partial-sum scratch too small for this block"};
  return (int)c;
}
constexpr int kColTile = 16;
constexpr int kColFused = 32;  // widest one-wavefront fused pass
}  // namespace

template <typename T>
void col_dots(QView<const T> Q, int ma, int vcol, const int* pmask,
              const double* dscale, int64_t nrows, double* C, Partials& P,
              hipStream_t st) {
  if (ma <= 0) return;
  const int64_t npanels = nrows / kPanel;
  // column tile: 1, 4 or 8 columns for the first steps (no loads of
  // absent columns), 16 beyond
  const int ct = ma <= 1 ? 1 : (ma <= 4 ? 4 : (ma <= 8 ? 8 : kColTile));
  const int ctiles = (ma + ct - 1) / ct;
  const int chunks = col_chunks(npanels, ctiles, ma, P);
  if (ct == 1)
    hipLaunchKernelGGL((k_col_dots<T, 1>), dim3(chunks * ctiles),
                       dim3(kBlock), 0, st, Q, ma, vcol, pmask, npanels,
                       ctiles, chunks, P.buf);
  else if (ct == 4)
    hipLaunchKernelGGL((k_col_dots<T, 4>), dim3(chunks * ctiles),
                       dim3(kBlock), 0, st, Q, ma, vcol, pmask, npanels,
                       ctiles, chunks, P.buf);
  else if (ct == 8)
    hipLaunchKernelGGL((k_col_dots<T, 8>), dim3(chunks * ctiles),
                       dim3(kBlock), 0, st, Q, ma, vcol, pmask, npanels,
                       ctiles, chunks, P.buf);
  else
    hipLaunchKernelGGL((k_col_dots<T, kColTile>), dim3(chunks * ctiles),
                       dim3(kBlock), 0, st, Q, ma, vcol, pmask, npanels,
                       ctiles, chunks, P.buf);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(kRedThreads), 0, st,
                     (const double*)P.buf, (int64_t)chunks, ma, 0, pmask,
                     dscale, C, (double*)nullptr, (double*)nullptr,
                     (int*)nullptr, 0);
  SGM_CHECK_LAUNCH();
}

template <typename T>
void col_update(QView<T> Q, int ma, int vcol, const double* w,
                const double* vscale, const int* pmask, int64_t nrows,
                double* R, double* Rinv, int* p_out, Partials& P,
                hipStream_t st) {
  const int64_t npanels = nrows / kPanel;
  const int chunks = col_chunks(npanels, 1, 1, P);
  const size_t lds = sizeof(T) * (size_t)(ma > 0 ? ma : 1);
  hipLaunchKernelGGL(k_col_update<T>, dim3(chunks), dim3(kBlock), lds, st, Q,
                     ma, vcol, w, vscale, pmask, npanels, chunks, P.buf);
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(kRedThreads), 0, st,
                     (const double*)P.buf, (int64_t)chunks, 0, 1, pmask,
                     (const double*)nullptr, (double*)nullptr, R, Rinv,
                     p_out, 0);
  SGM_CHECK_LAUNCH();
}

template <typename T>
bool col_update_dots(QView<T> Q, int ma, int vcol, const double* w,
                     int64_t nrows, double* R, double* Rinv, int* p_out,
                     double* C, Partials& P, hipStream_t st) {
  if (ma < 1 || ma > kColWideMax) return false;
  const int64_t npanels = nrows / kPanel;
  const int chunks = col_chunks(npanels, 1, ma + 1, P);
  if (ma > kColFused) {
    const int nwv = (ma + kColWave - 1) / kColWave;
    hipLaunchKernelGGL(k_col_update_dots_wide<T>, dim3(chunks),
                       dim3(nwv * kWave), 0, st, Q, ma, vcol, w, npanels,
                       chunks, P.buf);
  } else {
#define SGM_CUD(MA)                                                       \
  hipLaunchKernelGGL((k_col_update_dots<T, MA>), dim3(chunks), dim3(kBlock), \
                     0, st, Q, ma, vcol, w, npanels, chunks, P.buf)
  if (ma <= 4)
    SGM_CUD(4);
  else if (ma <= 8)
    SGM_CUD(8);
  else if (ma <= 16)
    SGM_CUD(16);
  else
    SGM_CUD(32);
#undef SGM_CUD
  }
  SGM_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(kRedThreads), 0, st,
                     (const double*)P.buf, (int64_t)chunks, ma, 1,
                     (const int*)nullptr, (const double*)nullptr, C, R, Rinv,
                     p_out, 1);
  SGM_CHECK_LAUNCH();
  return true;
}

template <typename T>
void col_scale(QView<T> Q, int vcol, const double* z, const int* pmask,
               int64_t nrows, hipStream_t st) {
  int64_t grid = ceil_div(nrows, kBlock);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_col_scale<T>, dim3((unsigned)grid), dim3(kBlock), 0, st,
                     Q, vcol, z, pmask, nrows);
  SGM_CHECK_LAUNCH();
}

#define SGM_INST(T)                                                          \
  template void gemm_tn<T>(QView<const T>, int, int, int, int, const int*,   \
                           int64_t, double*, int, Partials&, hipStream_t);   \
  template void update_gram<T>(QView<T>, int, int, int, int, const double*,  \
                               int, const int*, int64_t, double*, int,       \
                               Partials&, hipStream_t);                      \
  template void trsm_inv<T>(QView<T>, int, int, const double*, int,          \
                            const int*, int64_t, hipStream_t);               \
  template bool trsm_inv_gram<T>(QView<T>, int, int, const double*, int,     \
                                 const int*, int64_t, double*, int,          \
                                 Partials&, hipStream_t);                    \
  template void gemv_update<T>(QView<const T>, const double*, int,           \
                               const double*, double*, int64_t, hipStream_t); \
  template void col_dots<T>(QView<const T>, int, int, const int*,            \
                            const double*, int64_t, double*, Partials&,      \
                            hipStream_t);                                    \
  template void col_update<T>(QView<T>, int, int, const double*,             \
                              const double*, const int*, int64_t, double*,   \
                              double*, int*, Partials&, hipStream_t);        \
  template void col_scale<T>(QView<T>, int, const double*, const int*,       \
                             int64_t, hipStream_t);                          \
  template bool col_update_dots<T>(QView<T>, int, int, const double*,       \
                                   int64_t, double*, double*, int*, double*, \
                                   Partials&, hipStream_t);                  \
  template bool trsm_proj<T>(QView<T>, int, int, int, const double*, int,    \
                             const int*, int64_t, double*, int, Partials&,   \
                             hipStream_t);                                   \
  template void update_trsm<T>(QView<T>, int, int, int, const double*, int,  \
                               const double*, int, const int*, int64_t,      \
                               hipStream_t);
SGM_INST(double)
SGM_INST(float)
#undef SGM_INST

}  // namespace sgm
