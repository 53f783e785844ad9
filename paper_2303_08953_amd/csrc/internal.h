// Internal declarations shared by the HIP sources of the s-step GMRES
// library (gfx950, wave64).  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/sgm.h"

namespace sgm {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kSlice = 64;      // SELL-C slice height = one wavefront
constexpr int kLdAlign = 64;    // leading dimensions are multiples of this
constexpr int kSmallLds = 128;  // small FP64 matrices up to this size in LDS

// ------------------------------------------------------------------ errors
struct Error {
  sgm_status st;
  std::string msg;
};
void set_error(const std::string& m);
const char* last_error();

#define SGM_HIP(call)                                                      \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      throw ::sgm::Error{SGM_EHIP, std::string(#call) + ": " +             \
                                       hipGetErrorString(e_)};             \
  } while (0)

#define SGM_CHECK_LAUNCH() SGM_HIP(hipGetLastError())

#define SGM_REQUIRE(cond, msg)                                             \
  do {                                                                     \
    if (!(cond)) throw ::sgm::Error{SGM_EINVAL, (msg)};                    \
  } while (0)

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ layout
// Layout of a tall block of vectors (the Krylov basis Q).  Element (r, c)
// sits at base + (r >> plog) * pstride + c * cstride + (r & pmask):
//  - row panels (the solver's layout): 64-row panels, each holding the 64
//    rows of every column contiguously (plog = 6, cstride = 64,
//    pstride = 64 * ncols).  A kernel streaming many columns then reads a
//    few contiguous regions instead of one far-apart stream per column,
//    which keeps the memory system near its streaming bandwidth;
//  - column-major with leading dimension ld (one panel: plog = 62,
//    pstride = 0, cstride = ld), used by the step-level entry points.
// Rows are processed in aligned groups of 16 that never straddle a panel.
constexpr int kPanel = 64;
template <typename T>
struct QView {
  T* base = nullptr;
  int64_t pstride = 0;
  int64_t cstride = 0;
  int plog = 62;
  __host__ __device__ __forceinline__ int64_t row_off(int64_t r) const {
    return (r >> plog) * pstride + (r & ((int64_t(1) << plog) - 1));
  }
  __host__ __device__ __forceinline__ T* at(int64_t r, int64_t c) const {
    return base + row_off(r) + c * cstride;
  }
  __host__ __device__ __forceinline__ T* col(int64_t c) const {
    return base + c * cstride;
  }
  template <typename U>
  __host__ __device__ QView<U> as() const {
    QView<U> v;
    v.base = base;
    v.pstride = pstride;
    v.cstride = cstride;
    v.plog = plog;
    return v;
  }
};
template <typename T>
inline QView<T> panel_view(T* base, int ncols) {
  QView<T> v;
  v.base = base;
  v.pstride = (int64_t)kPanel * ncols;
  v.cstride = kPanel;
  v.plog = 6;
  return v;
}
template <typename T>
inline QView<T> colmajor_view(T* base, int64_t ld) {
  QView<T> v;
  v.base = base;
  v.pstride = 0;
  v.cstride = ld;
  v.plog = 62;
  return v;
}

// ------------------------------------------------------------------ matrix
// SELL-C sparse layout with C = 64 (one wavefront per slice of 64 rows).
// Slice s covers rows [64 s, 64 s + 64); its entries sit at
// ptr[s] + w * 64 + lane for w < width[s]; padding has val 0 and a column
// index that is already being read by the same lane (no extra traffic).
// Every ptr[s] is a multiple of 64, so ptr[s] / 64 + w numbers the
// (slice, position) groups of 64 entries.
struct Sell {
  int64_t n = 0;
  int64_t nslices = 0;
  int64_t nnz_padded = 0;
  int64_t* ptr = nullptr;   // [nslices + 1]
  int32_t* width = nullptr; // [nslices]
  int32_t* col = nullptr;   // [nnz_padded]
  // 16-bit relative columns, present when they fit (then the SpMV reads
  // these 2-byte offsets instead of the 4-byte columns): the entry of lane l
  // in group g = ptr[s] / 64 + w has column kbase[g] + l + rcol[entry].
  // kbase[g] is the midpoint of (column - lane) over the group's real rows,
  // so a group fits when that range spans at most 65535 (stencils of any
  // grid size, banded matrices); rows past n decode to a valid column.
  int16_t* rcol = nullptr;  // [nnz_padded]
  int32_t* kbase = nullptr; // [nnz_padded / 64]
  int64_t* src = nullptr;   // [nnz_padded] CSR index of each entry, -1 = pad
  double* val64 = nullptr;  // [nnz_padded]
  float* val32 = nullptr;   // [nnz_padded]
};

// ILU(0) factors (right preconditioner M = L U, zero fill-in).  Each
// substitution's rows are grouped by level (one more than the highest level
// among the rows the row depends on) and sorted within a level; the strict
// triangle of each position's row is stored in level order as ELL (entry t
// of position p at t * n + p; cnt[p] entries).
struct IluLevels {
  int32_t nlev = 0;           // levels (host copy)
  int32_t width = 0;          // largest row of the triangle (host copy)
  int32_t wpad = 0;           // ELL columns stored (>= width)
  int32_t max_level = 0;      // rows of the largest level (host copy)
  int32_t* rows = nullptr;    // [n] rows in level order
  int32_t* lptr = nullptr;    // [nlev + 1] first position of each level
  int32_t* cnt = nullptr;     // [n]
  int32_t* ecol = nullptr;    // [wpad * n]
  int32_t* epos = nullptr;    // [wpad * n] the column's level-order position
  int32_t* esrc = nullptr;    // [wpad * n] CSR index of the entry, -1 pad
  double* eval = nullptr;     // [wpad * n] factor values, 0 in the padding
};
struct Ilu {
  int32_t* dpos = nullptr;     // [n] CSR index of each diagonal entry
  double* fac = nullptr;       // [nnz] L (strict lower) and U, CSR order
  double* dinv = nullptr;      // [n] 1 / u_rr in backward-level order
  int32_t* nlev_dev = nullptr; // [4] levels of the forward, backward side;
                               // far flags of each (solve: LDS-only barrier
                               // when 0)
  int32_t* flags = nullptr;    // [4] analysis / pivot flags
  IluLevels L, U;
  int32_t max_level = 0;       // rows of the largest level, both sides
  int32_t* l2u = nullptr;      // [n] backward position of each forward one
  double* tl = nullptr;        // [n] solve scratch (forward level order)
  double* tu = nullptr;        // [n] solve scratch (backward level order)
  bool ok = false;             // factors valid for the current values
};

struct Matrix {
  int64_t n = 0, nnz = 0;
  int32_t* row_ptr = nullptr;  // CSR copy (device)
  int32_t* col = nullptr;
  int32_t* row_of = nullptr;   // row index of every nonzero
  double* val = nullptr;       // current values, CSR order
  double* diag = nullptr;      // [n]
  int64_t bandwidth = 0;       // max |column - row| over the nonzeros
  Sell fwd;                    // A
  Sell trn;                    // A^T
  Ilu* ilu = nullptr;          // ILU(0) factors, built on request
  // Jacobi-scaled value copies (A D^{-1}), built on demand inside a solve's
  // workspace; nothing cached here.
};

Matrix* matrix_create(int64_t n, int64_t nnz, const int32_t* row_ptr,
                      const int32_t* col, const double* val, hipStream_t st);
void matrix_update_values(Matrix* M, const double* val, hipStream_t st);
void matrix_destroy(Matrix* M);

void sell_build(Sell& S, int64_t n, const int32_t* row_ptr,
                const int32_t* col, const int32_t* perm_or_null,
                hipStream_t st);
void sell_fill_values(const Sell& S, const double* csr_val, hipStream_t st);
void sell_free(Sell& S);
void matrix_extract_diag(Matrix& M, hipStream_t st);

// ILU(0): analysis (diagonal positions, levels, level-ordered structure)
// and factorisation; ilu_factor recomputes the factors from the current
// values.  Both throw SGM_EINVAL (no stored diagonal, unsorted columns) or
// SGM_ENUMERIC (zero or non-finite pivot).
void ilu_build(Matrix& M, hipStream_t st);
void ilu_factor(Matrix& M, hipStream_t st);
void ilu_free(Ilu*& I);
// z = M^{-1} b (float64), b read at BV.row_off(row); b may be z.
void ilu_apply(const Ilu& I, int64_t n, QView<const double> BV,
               const double* b, double* z, hipStream_t st);

// ------------------------------------------------------------------ SpMV
enum SpmvEpi { EPI_PLAIN = 0, EPI_MPK = 1, EPI_RESID = 2 };

// y = A x on SELL values `val` (float64 or float32); scale[] (optional,
// per column) multiplies the value: A D^{-1} when scale = 1/diag.
template <typename T>
void spmv_plain(const Sell& S, const T* val, const T* x, T* y,
                hipStream_t st);
// y = ((A x) - theta x - delta xprev) / gamma with (theta, gamma, delta) =
// rec[3 j .. 3 j + 2] read on the device.
// With gate given, the launch does nothing unless *gate == expect (read on
// the device when the kernel starts).
template <typename T>
void spmv_mpk(const Sell& S, const T* val, QView<T> Q, int jx, int jprev,
              int jy, const double* rec, int j, hipStream_t st,
              const int* gate = nullptr, int expect = 0);
// The same step with the fused square-sum epilogue: *norm2 = the float64
// sum of the stored y(r)^2; part holds spmv_grid(S) doubles (the number of
// SpMV workgroups, resid_partials(S)).
template <typename T>
void spmv_mpk_norm(const Sell& S, const T* val, QView<T> Q, int jx, int jprev,
                   int jy, const double* rec, int j, double* part,
                   double* norm2, hipStream_t st);
// The same step with a right preconditioner: y = ((A z) - theta x -
// delta xprev) / gamma, z = M^{-1} x given as a plain vector (float64).
void spmv_mpk_prec(const Sell& S, const double* val, QView<double> Q,
                   const double* z, int jx, int jprev, int jy,
                   const double* rec, int j, hipStream_t st);
// x(0:n) += z(0:n) (float64)
void axpy_f64(const double* z, double* x, int64_t n, hipStream_t st);
// Depth-k matrix powers kernel (temporal blocking over row slabs): the
// steps j of one block, each y = column ycol from x = column xcol (and the
// previous vector, column pcol, when pcol >= 0) with records rec[3 j..].
struct MpkStep {
  int xcol, pcol, ycol, j;
};
constexpr int kMaxMpkTasks = 4;  // deepest fusion (steps per pass)
struct MpkTask {
  int64_t s0, ns;  // slices [s0, s0 + ns)
  int xcol, pcol, ycol, j;
};
struct MpkTasks {
  MpkTask t[kMaxMpkTasks];
  int wg[kMaxMpkTasks + 1];  // first workgroup of each piece (multiples of 8)
  int count;
};
struct MpkPlan {
  int depth = 1;             // steps per pass over the matrix (1 = unfused)
  int64_t slab_slices = 0;   // slices per row slab
  int64_t nslabs = 0;
};
// The slab plan for a depth (falls back to depth 1 when the matrix has
// fewer than three slabs of at least its bandwidth).
MpkPlan mpk_plan(const Sell& S, int64_t bandwidth, int depth, int vbytes);
template <typename T>
void spmv_mpk_steps(const Sell& S, const T* val, QView<T> Q,
                    const MpkStep* steps, int nsteps, const double* rec,
                    const MpkPlan& plan, hipStream_t st);
// r = b - A x (float64) and per-block partial sums of r^2 into part[];
// returns the number of partials written.
int64_t spmv_resid(const Sell& S, const double* val, const double* x,
                   const double* b, double* r, double* part, hipStream_t st);
int64_t resid_partials(const Sell& S);

// ------------------------------------------------------------------ vectors
// out[0] = sqrt(sum part[0..np)) (deterministic order).
void reduce_norm(const double* part, int64_t np, double* out, hipStream_t st);
// column c of Q = (T)(r / *beta) for rows < n, zero for rows n..ld-1.
template <typename T>
void scale_into(const double* r, const double* beta, QView<T> Q, int c,
                int64_t n, int64_t ld, hipStream_t st);
// zero rows n..ld-1 of columns [0, ncols) of Q
template <typename T>
void zero_pad_rows(QView<T> Q, int64_t n, int64_t ld, int ncols,
                   hipStream_t st);
void jacobi_values(const Matrix& M, const Sell& S, double* v64, float* v32,
                   hipStream_t st);
void vec_scale_div(double* x, const double* d, int64_t n, bool divide,
                   hipStream_t st);
void grad_vals(const Matrix& M, const double* lam, const double* x,
               double* g, hipStream_t st);
void cast_f64_f32(const double* a, float* b, int64_t n, hipStream_t st);
void copy_f64(const double* a, double* b, int64_t n, hipStream_t st);

// ------------------------------------------------------------------ tall-skinny
// Partial-sum scratch for the grid reductions.
struct Partials {
  double* buf = nullptr;
  int64_t cap = 0;  // doubles
};

// C(ma x nb, ld ldc, float64) = Q(:, a0:a0+ma)^T Q(:, b0:b0+nb) over rows
// [0, nrows).  ncount (device, may be NULL) masks the B columns: only
// min(nb, *ncount) are used (the rest of C is written as zero).
template <typename T>
void gemm_tn(QView<const T> Q, int a0, int ma, int b0, int nb,
             const int* ncount, int64_t nrows, double* C, int ldc,
             Partials& P, hipStream_t st);

// Q(:, b0:b0+nc) -= Q(:, a0:a0+ka) M(0:ka, 0:nc) (M float64, column-major,
// ld ldm) and, when G is not NULL, G(nc x nc, ld ldg) = the Gram matrix of
// the updated columns.  ncount (device, may be NULL) limits nc.
template <typename T>
void update_gram(QView<T> Q, int a0, int ka, int b0, int nc, const double* M,
                 int ldm, const int* ncount, int64_t nrows, double* G,
                 int ldg, Partials& P, hipStream_t st);

// Q(:, b0:b0+p) = Q(:, b0:b0+p) Rinv(0:p, 0:p) in place (Rinv upper
// triangular, float64, ld ldr), p = min(s, *pcount).
template <typename T>
void trsm_inv(QView<T> Q, int b0, int s, const double* Rinv, int ldr,
              const int* pcount, int64_t nrows, hipStream_t st);

// x(0:n) += scale * Q(:, 0:k) y(0:k), x float64, Q float64/float32,
// scale read from sdev (NULL = 1).
template <typename T>
void gemv_update(QView<const T> Q, const double* y, int k,
                 const double* sdev, double* x, int64_t n, hipStream_t st);

// Fused Q(:, b0:b0+p) = V Zinv (in place, p = min(nc, *pcount)) and
// R2 (ka x nc, ld ldr) = Q(:, 0:ka)^T Q(:, b0:b0+p) (columns >= p zero).
// Returns false (and does nothing) for shapes it does not cover (float32,
// ka > 64, nc > 32 or nc < 2); the caller then runs trsm_inv + gemm_tn.
template <typename T>
bool trsm_proj(QView<T> Q, int ka, int b0, int nc, const double* Zinv,
               int ldz, const int* pcount, int64_t nrows, double* R2, int ldr,
               Partials& P, hipStream_t st);

// trsm_inv plus the Gram of the result, G (s x s, ld ldg, symmetric) =
// Q(:, b0:b0+p)^T Q(:, b0:b0+p), zero outside p = min(s, *pcount).  Returns
// false (and does nothing) beyond 64 columns.
template <typename T>
bool trsm_inv_gram(QView<T> Q, int b0, int s, const double* Rinv, int ldr,
                   const int* pcount, int64_t nrows, double* G, int ldg,
                   Partials& P, hipStream_t st);

// Second pass of the Pythagorean BCGS2 variant in one pass over the block:
// Q(:, b0:b0+p) = (Q(:, b0:b0+p) - Q(:, 0:ka) M(0:ka, 0:p)) Zinv(0:p, 0:p),
// p = min(nc, *pcount), M ld ldm, Zinv upper triangular ld ldz.
template <typename T>
void update_trsm(QView<T> Q, int ka, int b0, int nc, const double* M,
                 int ldm, const double* Zinv, int ldz, const int* pcount,
                 int64_t nrows, hipStream_t st);

// G2 (nc x nc, ld ldg) = Gk - R2^T R2 on the leading p1 = min(nc, *pcount)
// block, zero elsewhere, from C = [R2; Gk] ((ka + nc) x nc, ld ldc, Gk read
// on and above the diagonal).  Float64.
void pyth_gram(const double* C, int ldc, int ka, int nc, const int* pcount,
               double* G2, int ldg, hipStream_t st);

// One-column blocks (s = 1), nrows a multiple of the 64-row panel:
// C(0:ma) = Q(:, 0:ma)^T v with v = Q(:, vcol), times *dscale
// when given; pmask (device, may be NULL): zero result when *pmask == 0.
template <typename T>
void col_dots(QView<const T> Q, int ma, int vcol, const int* pmask,
              const double* dscale, int64_t nrows, double* C, Partials& P,
              hipStream_t st);
// v = v * (*vscale) - Q(:, 0:ma) w (vscale may be NULL: no scaling), then
// Alg. 3 on the 1 x 1 Gram g = v^T v: *p_out = 1, R[0] = sqrt(g),
// Rinv[0] = 1 / R[0] when g > 0 is finite, else 0 and R, Rinv untouched.
// With *pmask == 0 (pmask may be NULL) nothing changes and *p_out = 0.
template <typename T>
void col_update(QView<T> Q, int ma, int vcol, const double* w,
                const double* vscale, const int* pmask, int64_t nrows,
                double* R, double* Rinv, int* p_out, Partials& P,
                hipStream_t st);
// The first CGS update of a one-column block fused with the second
// projection: v' = v - Q(:, 0:ma) w (as col_update without vscale/pmask),
// Alg. 3 on g = v'^T v' (p_out, R, Rinv as col_update), and
// C(0:ma) = Q(:, 0:ma)^T v' / R[0] (zero when *p_out = 0), i.e. what
// col_dots(Q, ma, vcol, p_out, Rinv, ...) gives after col_update, from one
// pass over Q(:, 0:ma).  Returns false, enqueueing nothing, when ma is
// outside [1, 256]; the caller then takes the two separate passes.
template <typename T>
bool col_update_dots(QView<T> Q, int ma, int vcol, const double* w,
                     int64_t nrows, double* R, double* Rinv, int* p_out,
                     double* C, Partials& P, hipStream_t st);
// v *= *z when *pmask > 0.
template <typename T>
void col_scale(QView<T> Q, int vcol, const double* z, const int* pmask,
               int64_t nrows, hipStream_t st);

// ------------------------------------------------------------------ small FP64
// Control block shared by the single-workgroup kernels of one block.
enum Ctrl {
  C_P1 = 0, C_P2, C_PH, C_BREAK, C_KDONE, C_CONV, C_BAD, C_NCTRL
};
// Device-only word after the control block: set by a block tail that ends
// a cycle (convergence, breakdown or a non-finite estimate) when the host
// has queued further steps without waiting; later tails then do nothing.
constexpr int C_STOP = C_NCTRL;
// Device-only word written by every block tail: the accepted size p2 when
// the cycle goes on, -1 when it ends.  Matrix powers steps of the next
// block queued before the host has seen the tail's result carry the size
// they assume and do nothing unless it matches.
constexpr int C_GO = C_NCTRL + 1;
constexpr int kCtrlWords = C_NCTRL + 2;

void pchol_ice(const double* G, int ldg, int smax, const int* s_dev,
               double omega, double* R, double* Rinv, int ldr, int* p_out,
               double* scratch, hipStream_t st);
void combine_r(const double* W, int ldw, const double* R2, int ldr2,
               const double* Z, const double* Zt, int ldz, int i,
               int* ctrl, double* Rtop, int ldt, double* Rkk, int ldk,
               hipStream_t st);
// Per-block tail of the solver: combine_r, Hessenberg recovery, Givens
// rotations and the convergence test in one single-workgroup kernel;
// Rtop / Rkk (may be NULL) receive R(1:nb, k) (ld ldw) and R(k, k) (ld ldz).
// res_out receives the per-column residual estimates and host_ctrl (may be
// NULL) a copy of the control words; both may point into host memory
// mapped for the device, so the host reads them without a copy.  stop (may
// be NULL, device): when *stop is set the tail does nothing; a tail that
// ends the cycle sets it (for steps queued ahead of the host's checks).
// seq > 0 (with host_ctrl): written last to host_ctrl[kSeqWord], after a
// system-scope fence, so the host can wait for the tail by polling that
// word instead of an event or a stream query.
constexpr int kSeqWord = 16;
size_t block_tail_scratch_doubles(int nb_max, int s_max);
void block_tail(const double* W, const double* R2, int ldw, const double* Z,
                const double* Zt, const double* Zi, const double* Zti, int ldz,
                int nb, int* ctrl, double* Rtop, double* Rkk, double* Hraw,
                double* Hr, int ldh, double* cs, double* sn, double* g,
                const double* rec, int n_rec, const double* beta0, double tol,
                double* res_out, int* host_ctrl, double* scratch,
                hipStream_t st, int* stop = nullptr, int seq = 0);
void back_solve(const double* Hr, int ldh, const double* g, const int* kdev,
                int kmax, double* y, hipStream_t st);
void givens_init(double* g, int m, const double* beta, hipStream_t st);

// Ritz values, Leja order, recurrence records, estimator.
void hqr_eigen(const double* H, int ldh, int m0, double* wr, double* wi,
               double* scratch, int* status, hipStream_t st);
void leja_records(const double* wr, const double* wi, int m0, int basis,
                  double eps, double omega_est, double* ritz_out,
                  double* rec, int* info_out, double* scratch,
                  hipStream_t st);
size_t shifts_scratch_doubles(int m0);

}  // namespace sgm
