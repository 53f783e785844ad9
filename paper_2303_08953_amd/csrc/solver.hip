// Host engine of the adaptive s-step GMRES (Alg. 4 with restarts, the Ritz
// pre-phase and estimator of Secs. 3.4-3.5, float32 inner cycles inside
// float64 refinement) and the C ABI.  Every arithmetic step runs in the HIP
// kernels of this library; the host only sequences launches, carves the
// caller's workspace and reads back the accepted block size and the
// convergence flags once per block.
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace sgm {

thread_local std::string g_last_error;
void set_error(const std::string& m) { g_last_error = m; }
const char* last_error() { return g_last_error.c_str(); }

namespace {

// ------------------------------------------------------------------ arena
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (size_t)(count > 0 ? count : 1);
    return p;
  }
};

struct Work {
  void* Q = nullptr;
  double* r = nullptr;
  double* jac64 = nullptr;
  float* jac32 = nullptr;
  double* ilu_z = nullptr;  // M^{-1} of the current vector (ILU(0))
  Partials P;
  double *W = nullptr, *G = nullptr, *Z = nullptr, *Zinv = nullptr;
  double *R2 = nullptr, *G2 = nullptr, *Zt = nullptr, *Ztinv = nullptr;
  double *Rtop = nullptr, *Rkk = nullptr;
  double *Hraw = nullptr, *Hr = nullptr, *cs = nullptr, *sn = nullptr;
  double *g = nullptr, *y = nullptr, *res_blk = nullptr;
  double *rec = nullptr, *mono = nullptr;
  double *wr = nullptr, *wi = nullptr, *ritz = nullptr;
  double *hqr_scr = nullptr, *leja_scr = nullptr, *pchol_scr = nullptr;
  double* tail_scr = nullptr;
  double* scal = nullptr;  // 0 beta0, 1 beta (current), 2 one
  int* ctrl = nullptr;     // C_NCTRL
  int* info = nullptr;     // 0 hqr status, 1..3 leja info
  int64_t ld = 0;
  int qcols = 0;  // columns of the basis panels (>= m + 2)
  int ldw = 0, lds = 0, ldh = 0;
};

// Columns of the basis panels: at least m + 2, skipping counts whose panel
// stride (64 rows x columns x value bytes) lies within 2 KiB of a multiple
// of 64 KiB.  Measured on the matrix powers SpMV, whose x gathers and y
// stores hop from panel to panel: such strides (128 or 254-258 float64
// columns, 254-258 or 512 float32 columns) slow it by 15-50%, on 2D and 3D
// stencils alike; the strides around them run at full speed.
int basis_cols(int m, int vb) {
  int c = m + 2;
  for (;;) {
    const int64_t rem = (int64_t)kPanel * c * vb % 65536;
    if ((rem < 65536 - rem ? rem : 65536 - rem) >= 2048) return c;
    ++c;
  }
}

// Partial sums of the grid reductions: room for 512 row chunks of the
// widest product ((m + 1) x s_max), so the products of wide blocks keep two
// workgroups per CU (fewer chunks when n has fewer 64-row panels).
int64_t part_cap(int m, int smax, int64_t n) {
  int64_t chunks = n / kPanel;
  chunks = chunks < 8 ? 8 : (chunks > 512 ? 512 : chunks);
  int64_t a = (int64_t)1 << 22;
  int64_t b = chunks * (m + 1) * smax;
  return a > b ? a : b;
}

void layout(Arena& a, Work& w, int64_t n, int64_t sell_nnz, int m, int smax,
            int nshift_max, bool fp32, bool jacobi, bool ilu) {
  w.ld = round_up(n, kLdAlign);
  w.ldw = m + 1;
  w.lds = smax;
  w.ldh = m + 1;
  w.qcols = basis_cols(m, fp32 ? 4 : 8);
  if (fp32)
    w.Q = a.take<float>(w.ld * w.qcols);
  else
    w.Q = a.take<double>(w.ld * w.qcols);
  w.r = a.take<double>(w.ld);
  if (jacobi) {
    w.jac64 = a.take<double>(sell_nnz);
    w.jac32 = a.take<float>(sell_nnz);
  }
  if (ilu) w.ilu_z = a.take<double>(w.ld);
  w.P.cap = part_cap(m, smax, n);
  w.P.buf = a.take<double>(w.P.cap);
  const int64_t ws = (int64_t)w.ldw * smax, ss = (int64_t)smax * smax;
  w.W = a.take<double>(ws);
  w.R2 = a.take<double>(ws);
  w.Rtop = a.take<double>(ws);
  w.G = a.take<double>(ss);
  w.G2 = a.take<double>(ss);
  w.Z = a.take<double>(ss);
  w.Zinv = a.take<double>(ss);
  w.Zt = a.take<double>(ss);
  w.Ztinv = a.take<double>(ss);
  w.Rkk = a.take<double>(ss);
  w.Hraw = a.take<double>((int64_t)w.ldh * m);
  w.Hr = a.take<double>((int64_t)w.ldh * m);
  w.cs = a.take<double>(m);
  w.sn = a.take<double>(m);
  w.g = a.take<double>(m + 1);
  w.y = a.take<double>(m + 1);
  w.res_blk = a.take<double>(smax + 1);
  const int nr = nshift_max > 0 ? nshift_max : 1;
  w.rec = a.take<double>(3 * nr);
  w.mono = a.take<double>(4);
  w.wr = a.take<double>(nr);
  w.wi = a.take<double>(nr);
  w.ritz = a.take<double>(2 * nr);
  w.hqr_scr = a.take<double>((int64_t)nr * nr);
  w.leja_scr = a.take<double>((int64_t)shifts_scratch_doubles(nr));
  w.pchol_scr = a.take<double>(2 * ss + 2 * smax);
  w.tail_scr = a.take<double>((int64_t)block_tail_scratch_doubles(m + 1, smax));
  w.scal = a.take<double>(8);
  w.ctrl = a.take<int>(kCtrlWords);
  w.info = a.take<int>(8);
}

// Pinned host memory, mapped for the device and coherent: the block tail
// writes the control words and residual estimates straight into it, and
// the host reads them once the stream is idle (no copy kernels).
struct HostMirror {
  int* ctrl = nullptr;      // host view
  double* res = nullptr;
  double* scal = nullptr;
  int* dctrl = nullptr;     // device views of the same bytes
  double* dres = nullptr;
  // one slot per queued column-wise step (control words, residual estimate)
  int* slot_ctrl = nullptr;
  double* slot_res = nullptr;
  int* dslot_ctrl = nullptr;
  double* dslot_res = nullptr;
};
constexpr size_t kSlotCtrlOff = 32 * 1024;  // kMaxSlots x kSlotInts ints
constexpr int kSlotInts = 8;
constexpr int kMaxSlots = 256;
constexpr int kStepBatch = 32;  // column-wise steps queued per synchronisation
constexpr size_t kSlotResOff =
    kSlotCtrlOff + sizeof(int) * kSlotInts * kMaxSlots;  // kMaxSlots doubles
static_assert(C_NCTRL <= kSlotInts, "control words do not fit a slot");

// Wait for the stream by polling: a blocking synchronisation sleeps and
// wakes up tens of microseconds late, once per block.
void wait_stream(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e == hipSuccess) return;
    if (e != hipErrorNotReady) {
      (void)hipGetLastError();
      throw Error{SGM_EHIP, std::string("stream: ") + hipGetErrorString(e)};
    }
  }
}

// Wait for the block tail with sequence number seq by polling the word it
// writes last into the mapped host memory.  (An event recorded behind the
// tail would do, but each event in the stream leaves the GPU idle for a
// few microseconds between kernels.)  Now and then the stream is queried,
// so that a failed launch ends the wait with its error.
void wait_seq(const int* word, int seq, hipStream_t st) {
  for (uint64_t it = 1;; ++it) {
    if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == seq) return;
    if ((it & 1023) == 0) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == seq) return;
        throw Error{SGM_EHIP, "block tail ended without its sequence word"};
      }
      if (e != hipErrorNotReady) {
        (void)hipGetLastError();
        throw Error{SGM_EHIP, std::string("stream: ") + hipGetErrorString(e)};
      }
    }
  }
}

// Matrix powers steps of the next block queued behind a block's tail,
// before the host has read the tail's result (the block size they assume
// is the one just used; gated on the device, see C_GO).  While the GPU
// runs them the host reads the result and queues the rest of the block,
// so the stream does not run dry once per block.
constexpr int kSpecSteps = 4;

struct Handle {
  Matrix* M = nullptr;
  void* pinned = nullptr;      // hipHostMalloc'd readback area (host view)
  void* pinned_dev = nullptr;  // the same memory as the device sees it
  size_t pinned_bytes = 0;
};

constexpr size_t kPinnedBytes = 64 * 1024;

double unit_roundoff(bool fp32) {
  return fp32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
}

double default_omega(bool fp32) { return 0.1 / std::sqrt(unit_roundoff(fp32)); }

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t).count();
}

// ------------------------------------------------------------------ block
// Block orthogonalisation of V = Q(:, nb : nb+s-1) against Q(:, 0 : nb-1):
// BCGS2 with two partial CholQR passes (Alg. 4).  The accepted
// sizes stay on the device (ctrl[C_P1], ctrl[C_P2]); later kernels read
// them, so the sequence needs no host synchronisation.
template <typename T>
void orth_block(QView<T> Q, int64_t nrows, int nb, int s, double omega,
                Work& w, hipStream_t st, bool combine = true,
                bool pyth = false) {
  const QView<const T> Qc = Q.template as<const T>();
  int* p1 = w.ctrl + C_P1;
  int* p2 = w.ctrl + C_P2;
  if (s == 1) {
    // One column (CGS2).  The first normalisation v / r1 is not stored: the
    // second projection is taken as (Q^T v) / r1 and the second update
    // scales v on the way.  With a scalar r1 this changes only the rounding.
    col_dots<T>(Qc, nb, nb, nullptr, nullptr, nrows, w.W, w.P, st);
    // up to 256 prior columns the first update and the second projection
    // share one pass over Q (the columns stay in registers in between)
    if (!col_update_dots<T>(Q, nb, nb, w.W, nrows, w.Z, w.Zinv, p1, w.R2,
                            w.P, st)) {
      col_update<T>(Q, nb, nb, w.W, nullptr, nullptr, nrows, w.Z, w.Zinv, p1,
                    w.P, st);
      col_dots<T>(Qc, nb, nb, p1, w.Zinv, nrows, w.R2, w.P, st);
    }
    col_update<T>(Q, nb, nb, w.R2, w.Zinv, p1, nrows, w.Zt, w.Ztinv, p2, w.P,
                  st);
    col_scale<T>(Q, nb, w.Ztinv, p2, nrows, st);
    if (combine)
      combine_r(w.W, w.ldw, w.R2, w.ldw, w.Z, w.Zt, w.lds, nb, w.ctrl, w.Rtop,
                w.ldw, w.Rkk, w.lds, st);
    return;
  }
  // first BCGS: W = Q^T V; V -= Q W; G = V^T V
  gemm_tn<T>(Qc, 0, nb, nb, s, nullptr, nrows, w.W, w.ldw, w.P, st);
  update_gram<T>(Q, 0, nb, nb, s, w.W, w.ldw, nullptr, nrows, w.G, w.lds,
                 w.P, st);
  // first partial CholQR: p1, Z; V(:, 0:p1) = V Z^{-1}
  pchol_ice(w.G, w.lds, s, nullptr, omega, w.Z, w.Zinv, w.lds, p1,
            w.pchol_scr, st);
  if (pyth) {
    // Pythagorean second pass: Q_1 = V Zinv with its Gram Gk from the
    // same registers, R2 = Q^T Q_1, stored as [R2; Gk] ((nb + s) x s, ld
    // ldw); G2 = Gk - R2^T R2; then (Q_1 - Q R2) Zt^{-1} in one pass.
    // Beyond 64 columns the Gram comes from one wider product instead.
    // (Fusing the projection into the triangular solve, as the classical
    // path does, measured slower here: the extra Gram accumulators cost
    // the kernel its occupancy.)
    if (w.ldw < nb + s)
      throw Error{SGM_EINVAL, "orth_block: R2 workspace too short"};
    if (trsm_inv_gram<T>(Q, nb, s, w.Zinv, w.lds, p1, nrows, w.R2 + nb,
                         w.ldw, w.P, st)) {
      gemm_tn<T>(Qc, 0, nb, nb, s, p1, nrows, w.R2, w.ldw, w.P, st);
    } else {
      trsm_inv<T>(Q, nb, s, w.Zinv, w.lds, p1, nrows, st);
      gemm_tn<T>(Qc, 0, nb + s, nb, s, p1, nrows, w.R2, w.ldw, w.P, st);
    }
    pyth_gram(w.R2, w.ldw, nb, s, p1, w.G2, w.lds, st);
    pchol_ice(w.G2, w.lds, s, p1, omega, w.Zt, w.Ztinv, w.lds, p2,
              w.pchol_scr, st);
    update_trsm<T>(Q, nb, nb, s, w.R2, w.ldw, w.Ztinv, w.lds, p2, nrows, st);
    if (combine)
      combine_r(w.W, w.ldw, w.R2, w.ldw, w.Z, w.Zt, w.lds, nb, w.ctrl, w.Rtop,
                w.ldw, w.Rkk, w.lds, st);
    return;
  }
  // V(:, 0:p1) = V Zinv, then the second BCGS projection R2 = Q^T V on
  // the p1 accepted columns (fused when the shape allows)
  if (!trsm_proj<T>(Q, nb, nb, s, w.Zinv, w.lds, p1, nrows, w.R2, w.ldw, w.P,
                    st)) {
    trsm_inv<T>(Q, nb, s, w.Zinv, w.lds, p1, nrows, st);
    gemm_tn<T>(Qc, 0, nb, nb, s, p1, nrows, w.R2, w.ldw, w.P, st);
  }
  update_gram<T>(Q, 0, nb, nb, s, w.R2, w.ldw, p1, nrows, w.G2, w.lds, w.P,
                 st);
  // second partial CholQR: p2, Zt; V(:, 0:p2) = V Zt^{-1}
  pchol_ice(w.G2, w.lds, s, p1, omega, w.Zt, w.Ztinv, w.lds, p2, w.pchol_scr,
            st);
  trsm_inv<T>(Q, nb, s, w.Ztinv, w.lds, p2, nrows, st);
  if (combine)
    combine_r(w.W, w.ldw, w.R2, w.ldw, w.Z, w.Zt, w.lds, nb, w.ctrl, w.Rtop,
              w.ldw, w.Rkk, w.lds, st);
}

struct Shifts {
  bool known = false;
  std::vector<double> rec;  // host copy, 3 per step
  int n_rec = 0;
  int s_init = 1;
  int s0 = 0;
  int hits = 0;
};

struct Result {
  int iters = 0, restarts = 0, outer = 0;
  double rel_true = 1.0, rel_est = 1.0;
  sgm_status status = SGM_NOT_CONVERGED;
  std::vector<double> res_hist;
  std::vector<int> s_hist;
  double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int s0 = 0, s_init = 0, n_rec = 0, hits = 0;
  int64_t n_spmv = 0;
  double t_spmv = 0.0;
  int mpk_depth = 1;
  int64_t mpk_slab_rows = 0;
};

template <typename T>
struct Engine {
  const Matrix& A;
  const Sell& S;
  const T* vals;        // values the inner cycles use (T precision)
  const double* vals64; // float64 values for true residuals
  Work& w;
  HostMirror hm;
  hipStream_t st;
  int64_t n, ld;
  int m;
  double omega;
  double eps;
  const sgm_opts& o;
  Shifts sh;
  Result& res;
  // Per block two events: the start and the end of its matrix powers steps
  // (two sets in turn: block k uses set k % 2).  A block's
  // orthogonalisation and tail take the time from its last step to the
  // next block's first; the cycle's last block ends at ecyc.
  hipEvent_t em0[2], em1[2], ecyc;
  int last = 1;             // set of the last block
  bool orth_open = false;   // a block of this cycle has run
  bool orth_pending = false;  // ecyc recorded, the last block's time unread
  int seq = 0;              // sequence number of the last block tail
  MpkPlan mplan;
  std::vector<MpkStep> msteps, spec_steps;
  const Ilu* ilu = nullptr;  // right ILU(0) preconditioner (float64 only)

  Engine(const Matrix& A_, const Sell& S_, const T* v, const double* v64,
         Work& w_, HostMirror hm_, hipStream_t st_, const sgm_opts& o_,
         Result& r_)
      : A(A_), S(S_), vals(v), vals64(v64), w(w_), hm(hm_), st(st_),
        n(A_.n), ld(w_.ld), m(o_.restart), o(o_), res(r_) {
    const bool f32 = sizeof(T) == 4;
    omega = o.omega > 0 ? o.omega : default_omega(f32);
    eps = unit_roundoff(f32);
    for (auto& e : em0) SGM_HIP(hipEventCreate(&e));
    for (auto& e : em1) SGM_HIP(hipEventCreate(&e));
    SGM_HIP(hipEventCreate(&ecyc));
    // earlier solves on this handle have finished: continue their sequence
    seq = std::max(0, __atomic_load_n(hm.ctrl + kSeqWord, __ATOMIC_ACQUIRE));
    mplan = mpk_plan(S, A.bandwidth, o.mpk_depth, (int)sizeof(T));
    res.mpk_depth = mplan.depth;
    res.mpk_slab_rows = mplan.depth > 1 ? mplan.slab_slices * kSlice : 0;
  }
  ~Engine() {
    for (auto& e : em0) (void)hipEventDestroy(e);
    for (auto& e : em1) (void)hipEventDestroy(e);
    (void)hipEventDestroy(ecyc);
  }

  // The last block's orthogonalisation time of the previous cycle (the
  // stream is idle when this runs: after the true residual).
  void flush_timing() {
    if (orth_pending) {
      SGM_HIP(hipEventSynchronize(ecyc));
      float to = 0;
      SGM_HIP(hipEventElapsedTime(&to, em1[last], ecyc));
      res.t[3] += to;
      orth_pending = false;
    }
    orth_open = false;
  }

  // the basis Q(:, 0 : m+1) in 64-row panels of w.qcols columns
  QView<T> Q() const { return panel_view<T>(static_cast<T*>(w.Q), w.qcols); }

  void set_monomial() {
    const double mono[3] = {0.0, 1.0, 0.0};
    SGM_HIP(hipMemcpyAsync(w.mono, mono, sizeof(mono), hipMemcpyHostToDevice,
                           st));
  }

  // Shifts from user-given Ritz values (skips the pre-phase).
  void shifts_from_host(const double* pairs, int ns) {
    SGM_HIP(hipMemcpyAsync(w.ritz, pairs, sizeof(double) * 2 * ns,
                           hipMemcpyHostToDevice, st));
    std::vector<double> re(ns), im(ns);
    for (int k = 0; k < ns; ++k) {
      re[k] = pairs[2 * k];
      im[k] = pairs[2 * k + 1];
    }
    SGM_HIP(hipMemcpyAsync(w.wr, re.data(), sizeof(double) * ns,
                           hipMemcpyHostToDevice, st));
    SGM_HIP(hipMemcpyAsync(w.wi, im.data(), sizeof(double) * ns,
                           hipMemcpyHostToDevice, st));
    wait_stream(st);
    finish_shifts(ns, false);
  }

  // Ritz values of the pre-phase Hessenberg H(0:m0, 0:m0), Leja order,
  // recurrence records and (scaled Newton) the estimator's s0*.
  void compute_shifts(int m0) {
    if (m0 <= 0) {
      // breakdown before any column: a single neutral record
      sh.rec = {0.0, 1.0, 0.0};
      sh.n_rec = 1;
      SGM_HIP(hipMemcpyAsync(w.rec, sh.rec.data(), sizeof(double) * 3,
                             hipMemcpyHostToDevice, st));
      sh.known = true;
      sh.s_init = o.s_max;
      return;
    }
    hqr_eigen(w.Hraw, w.ldh, m0, w.wr, w.wi, w.hqr_scr, w.info, st);
    finish_shifts(m0, true);
  }

  void finish_shifts(int m0, bool check_hqr) {
    const bool scaled = o.basis == SGM_BASIS_SCALED_NEWTON;
    const double om_est =
        (scaled && o.use_estimator)
            ? (o.omega_est > 0 ? o.omega_est : default_omega(sizeof(T) == 4))
            : 0.0;
    leja_records(w.wr, w.wi, m0, (int)o.basis, eps, om_est, w.ritz, w.rec,
                 w.info + 1, w.leja_scr, st);
    int info[4] = {0, 0, 0, 0};
    SGM_HIP(hipMemcpyAsync(info, w.info, sizeof(int) * 4,
                           hipMemcpyDeviceToHost, st));
    sh.rec.assign(3 * m0, 0.0);
    SGM_HIP(hipMemcpyAsync(sh.rec.data(), w.rec, sizeof(double) * 3 * m0,
                           hipMemcpyDeviceToHost, st));
    wait_stream(st);
    if ((check_hqr && info[0] != 0) || info[3] != 0)
      throw Error{SGM_ENUMERIC, "Ritz values: QR iteration failed or "
                                "non-finite values"};
    sh.known = true;
    sh.n_rec = m0;
    sh.s0 = info[1];
    sh.hits = info[2];
    sh.s_init = o.s_max;
    if (scaled && o.use_estimator && sh.s0 > 0)
      sh.s_init = std::max(1, std::min(o.s_max, sh.s0));
  }

  struct BlockOut {
    int p2, ph, brk, kdone, conv, bad;
  };

  // One matrix powers step with the right preconditioner: z = M^{-1} x,
  // then y = ((A z) - theta x - delta xprev) / gamma.
  void mpk_step_prec(const MpkStep& m, const double* rec) {
    if constexpr (sizeof(T) == 8) {
      const QView<double> Qd = Q();
      ilu_apply(*ilu, n, Qd.template as<const double>(), Qd.col(m.xcol),
                w.ilu_z, st);
      spmv_mpk_prec(S, vals, Qd, w.ilu_z, m.xcol, m.pcol, m.ycol, rec, m.j,
                    st);
    }
  }

  // The matrix powers steps of a block of s_eff columns from column nb.
  void make_steps(int nb, int s_eff, bool mono, std::vector<MpkStep>& out) {
    const int nrec = mono ? 1 : sh.n_rec;
    out.resize(s_eff);
    for (int j = 0; j < s_eff; ++j) {
      const int q = j % nrec;
      const double delta = mono ? 0.0 : sh.rec[3 * q + 2];
      const int jprev = (j >= 1 && delta != 0.0) ? nb - 2 + j : -1;
      out[j] = MpkStep{nb - 1 + j, jprev, nb + j, q};
    }
  }

  // One s-step block: MPK, BCGS2 + partial CholQR2, Hessenberg recovery,
  // Givens and the convergence test; one host synchronisation at the end.
  // The first `pre` matrix powers steps were queued by the previous block
  // (and found valid).  With spec_s > 0 the first steps of the next block
  // (spec_s columns from nb + s_eff, as if all s_eff columns are accepted)
  // are queued behind the tail before the host waits.
  BlockOut block(int nb, int s_eff, bool mono, const double* beta0,
                 double tol, int pre = 0, int spec_s = 0) {
    const double* rec = mono ? w.mono : w.rec;
    const int nrec = mono ? 1 : sh.n_rec;
    // this block's events; with steps queued ahead, their start event
    const int cur = last ^ 1;
    if (pre == 0) SGM_HIP(hipEventRecord(em0[cur], st));
    make_steps(nb, s_eff, mono, msteps);
    if (ilu != nullptr) {
      for (int j = 0; j < s_eff; ++j) mpk_step_prec(msteps[j], rec);
    } else {
      spmv_mpk_steps<T>(S, vals, Q(), msteps.data() + pre, s_eff - pre, rec,
                        mplan, st);
    }
    SGM_HIP(hipEventRecord(em1[cur], st));
    orth_block<T>(Q(), ld, nb, s_eff, omega, w, st, false,
                  o.orth == SGM_ORTH_BCGS2_PYTH);
    seq = seq >= INT_MAX - 1 ? 1 : seq + 1;
    block_tail(w.W, w.R2, w.ldw, w.Z, w.Zt, w.Zinv, w.Ztinv, w.lds, nb,
               w.ctrl, nullptr, nullptr, w.Hraw, w.Hr, w.ldh, w.cs, w.sn, w.g,
               rec, nrec, beta0, tol, hm.dres, hm.dctrl, w.tail_scr, st,
               nullptr, seq);
    if (spec_s > 0) {
      // the next block's first steps, gated on this block's result; they
      // start the next block's event set
      make_steps(nb + s_eff, spec_s, mono, spec_steps);
      SGM_HIP(hipEventRecord(em0[cur ^ 1], st));
      const int k = std::min(kSpecSteps, spec_s);
      for (int j = 0; j < k; ++j)
        spmv_mpk<T>(S, vals, Q(), spec_steps[j].xcol, spec_steps[j].pcol,
                    spec_steps[j].ycol, rec, spec_steps[j].j, st,
                    w.ctrl + C_GO, s_eff);
    }
    wait_seq(hm.ctrl + kSeqWord, seq, st);
    // the matrix powers steps of this block (with those queued ahead, and
    // any wait for the host between them), then the previous block's
    // orthogonalisation and tail
    float tm = 0;
    SGM_HIP(hipEventElapsedTime(&tm, em0[cur], em1[cur]));
    res.t[2] += tm;
    res.t_spmv += tm;
    res.n_spmv += s_eff;
    if (orth_open) {
      float to = 0;
      SGM_HIP(hipEventElapsedTime(&to, em1[last], em0[cur]));
      res.t[3] += to;
    }
    orth_open = true;
    last = cur;
    BlockOut b;
    b.p2 = hm.ctrl[C_P2];
    b.ph = hm.ctrl[C_PH];
    b.brk = hm.ctrl[C_BREAK];
    b.kdone = hm.ctrl[C_KDONE];
    b.conv = hm.ctrl[C_CONV];
    b.bad = hm.ctrl[C_BAD];
    return b;
  }

  // The column-wise pre-phase steps t0 + 1 .. t0 + nsteps (s = 1,
  // monomial), queued back to back with one host synchronisation at the
  // end (the stop word is cleared with the first batch): every step's
  // tail writes its control words and estimate into its own slot of the
  // mapped host memory, and the tail that ends the cycle (convergence,
  // breakdown, non-finite estimate) sets the device stop word, after which
  // the queued tails leave the Hessenberg and Givens state untouched (the
  // other kernels of those steps only touch columns the cycle no longer
  // uses).  Returns the slots' control words in order.
  std::vector<BlockOut> column_steps(int t0, int nsteps, const double* beta0,
                                     double tol) {
    if (t0 == 0) SGM_HIP(hipMemsetAsync(w.ctrl + C_STOP, 0, sizeof(int), st));
    for (int t = t0; t < t0 + nsteps; ++t) {
      const int nbt = 1 + t;
      if (ilu != nullptr)
        mpk_step_prec(MpkStep{nbt - 1, -1, nbt, 0}, w.mono);
      else
        spmv_mpk<T>(S, vals, Q(), nbt - 1, -1, nbt, w.mono, 0, st);
      orth_block<T>(Q(), ld, nbt, 1, omega, w, st, false);
      block_tail(w.W, w.R2, w.ldw, w.Z, w.Zt, w.Zinv, w.Ztinv, w.lds, nbt,
                 w.ctrl, nullptr, nullptr, w.Hraw, w.Hr, w.ldh, w.cs, w.sn,
                 w.g, w.mono, 1, beta0, tol, hm.dslot_res + t,
                 hm.dslot_ctrl + (size_t)kSlotInts * t, w.tail_scr, st,
                 w.ctrl + C_STOP);
    }
    wait_stream(st);
    std::vector<BlockOut> out;
    for (int t = t0; t < t0 + nsteps; ++t) {
      const int* c = hm.slot_ctrl + (size_t)kSlotInts * t;
      BlockOut b;
      b.p2 = c[C_P2];
      b.ph = c[C_PH];
      b.brk = c[C_BREAK];
      b.kdone = c[C_KDONE];
      b.conv = c[C_CONV];
      b.bad = c[C_BAD];
      out.push_back(b);
      if (b.bad || b.brk || b.conv || b.p2 == 0) break;
    }
    return out;
  }

  // One restart cycle from Q(:, 0) (already the normalised residual) with
  // g = beta_dev e_1.  Returns the number of Hessenberg columns and leaves
  // y in w.y.  res_scale converts the estimates to the caller's reference.
  int cycle(const double* beta_dev, const double* beta0_dev, double tol,
            bool prephase_only, double res_scale, bool* conv_out) {
    flush_timing();
    SGM_HIP(hipMemsetAsync(w.Hraw, 0, sizeof(double) * w.ldh * m, st));
    givens_init(w.g, m, beta_dev, st);
    const int m0 = sh.known ? 0 : std::min(o.s_max, m);
    const int last = prephase_only ? m0 : m;
    int nb = 1, k = 0, pre = 0;
    bool conv = false;
    int s = sh.s_init;
    // pre-phase block size: 1 (column-wise), or adaptive monomial blocks
    int s_pre = o.prephase == SGM_PREPHASE_MONOMIAL
                    ? std::max(1, std::min(o.prephase_s, std::max(m0, 1)))
                    : 1;
    auto t_pre = Clock::now();
    bool timing_pre = !sh.known;
    if (!sh.known && s_pre == 1 && m0 >= 1 && m0 <= kMaxSlots) {
      // the column-wise pre-phase, queued in batches without per-step
      // synchronisation (a batch bounds the steps queued past the end of
      // a cycle that converges early)
      for (int t0 = 0; t0 < m0 && !conv; t0 += kStepBatch) {
        const int cnt = std::min(kStepBatch, m0 - t0);
        const std::vector<BlockOut> bs =
            column_steps(t0, cnt, beta0_dev, prephase_only ? -1.0 : tol);
        for (size_t u = 0; u < bs.size(); ++u) {
          const BlockOut& b = bs[u];
          const size_t t = t0 + u;
          if (b.bad) throw Error{SGM_ENUMERIC, "non-finite residual estimate"};
          if (!prephase_only) {
            // one column per step: kdone is 0 or 1
            if (b.kdone > 0)
              res.res_hist.push_back(hm.slot_res[t] * res_scale);
            res.s_hist.push_back(b.brk ? 0 : b.p2);
            if (b.kdone > 0) res.rel_est = hm.slot_res[t] * res_scale;
          }
          k = nb - 1 + b.kdone;
          if (b.brk) {
            conv = true;
            break;
          }
          if (b.conv) conv = true;
          nb += b.p2;
          if (conv) break;
        }
      }
    }
    while (nb <= last && !conv) {
      if (!sh.known && nb > m0) {
        if (orth_open) {
          SGM_HIP(hipEventRecord(ecyc, st));
          orth_pending = true;
        }
        compute_shifts(nb - 1);  // waits for the stream
        flush_timing();
        s = sh.s_init;
        res.t[1] += ms_since(t_pre);
        timing_pre = false;
      }
      const bool in_pre = !sh.known;
      const int s_eff = in_pre ? std::min(std::min(s_pre, m0 + 1 - nb),
                                          m + 1 - nb)
                               : std::min(s, m + 1 - nb);
      // the next block's size if every column of this one is accepted
      int spec_s = 0;
      if (!in_pre && !prephase_only && ilu == nullptr && mplan.depth <= 1 &&
          nb + s_eff <= last)
        spec_s = std::min(s_eff, m + 1 - (nb + s_eff));
      BlockOut b = block(nb, s_eff, in_pre || o.basis == SGM_BASIS_MONOMIAL,
                         beta0_dev, prephase_only ? -1.0 : tol, pre, spec_s);
      pre = 0;
      if (b.bad) throw Error{SGM_ENUMERIC, "non-finite residual estimate"};
      if (!prephase_only) {
        for (int j = 0; j < b.kdone; ++j)
          res.res_hist.push_back(hm.res[j] * res_scale);
        res.s_hist.push_back(b.brk ? 0 : b.p2);
        if (b.kdone > 0) res.rel_est = hm.res[b.kdone - 1] * res_scale;
      }
      k = nb - 1 + b.kdone;
      if (b.brk) {
        conv = true;
        break;
      }
      if (b.conv) conv = true;
      nb += b.p2;
      if (!in_pre) s = b.p2;
      else if (o.prephase == SGM_PREPHASE_MONOMIAL) s_pre = b.p2;
      // the steps queued ahead are the next block's when all s_eff columns
      // were accepted and the cycle goes on (the device gate agrees)
      if (spec_s > 0 && !b.brk && !b.conv && !b.bad && b.p2 == s_eff)
        pre = std::min(kSpecSteps, spec_s);
    }
    if (orth_open) {
      SGM_HIP(hipEventRecord(ecyc, st));
      orth_pending = true;
    }
    if (!sh.known) {
      compute_shifts(k);
      if (timing_pre) res.t[1] += ms_since(t_pre);
    }
    if (conv_out) *conv_out = conv;
    if (prephase_only) return 0;
    back_solve(w.Hr, w.ldh, w.g, nullptr, k, w.y, st);
    return k;
  }
};

// ------------------------------------------------------------------ solve
template <typename T>
void run_solve(Handle* h, const double* b, const double* x0, double* x,
               const sgm_opts& o, Work& w, hipStream_t st, Result& R) {
  const Matrix& A = *h->M;
  const Sell& S = o.transpose ? A.trn : A.fwd;
  const int64_t n = A.n;
  const bool jac = o.precond == SGM_PRECOND_JACOBI;
  const bool ilu = o.precond == SGM_PRECOND_ILU0;
  const bool f32 = sizeof(T) == 4;
  if (ilu)
    SGM_REQUIRE(A.ilu != nullptr && A.ilu->ok,
                "no valid ILU(0) factors: call sgm_matrix_ilu0 first");
  auto t0 = Clock::now();
  HostMirror hm;
  hm.ctrl = static_cast<int*>(h->pinned);
  hm.res = reinterpret_cast<double*>(static_cast<char*>(h->pinned) + 256);
  hm.scal = reinterpret_cast<double*>(static_cast<char*>(h->pinned) + 128);
  hm.dctrl = static_cast<int*>(h->pinned_dev);
  hm.dres = reinterpret_cast<double*>(static_cast<char*>(h->pinned_dev) + 256);
  hm.slot_ctrl = reinterpret_cast<int*>(static_cast<char*>(h->pinned) +
                                        kSlotCtrlOff);
  hm.slot_res = reinterpret_cast<double*>(static_cast<char*>(h->pinned) +
                                          kSlotResOff);
  hm.dslot_ctrl = reinterpret_cast<int*>(static_cast<char*>(h->pinned_dev) +
                                         kSlotCtrlOff);
  hm.dslot_res = reinterpret_cast<double*>(
      static_cast<char*>(h->pinned_dev) + kSlotResOff);
  const double* v64 = S.val64;
  const float* v32 = S.val32;
  if (jac) {
    jacobi_values(A, S, w.jac64, w.jac32, st);
    v64 = w.jac64;
    v32 = w.jac32;
  }
  const T* vT;
  if constexpr (sizeof(T) == 4) vT = v32; else vT = v64;
  // x = x0 (or 0); with Jacobi the iterate is u = D x
  if (x0 == nullptr)
    SGM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
  else if (x0 != x)
    SGM_HIP(hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice,
                           st));
  if (jac) vec_scale_div(x, A.diag, n, false, st);
  zero_pad_rows<T>(panel_view<T>(static_cast<T*>(w.Q), w.qcols), n, w.ld,
                   o.restart + 2, st);
  const double one = 1.0;
  SGM_HIP(hipMemcpyAsync(w.scal + 2, &one, sizeof(double),
                         hipMemcpyHostToDevice, st));
  Engine<T> E(A, S, vT, v64, w, hm, st, o, R);
  if (ilu) {
    // one preconditioned step at a time (the fused kernel has no M^{-1})
    E.ilu = A.ilu;
    E.mplan = MpkPlan{};
    R.mpk_depth = 1;
    R.mpk_slab_rows = 0;
  }
  E.set_monomial();
  if (o.basis == SGM_BASIS_MONOMIAL) {
    E.sh.known = true;
    E.sh.rec = {0.0, 1.0, 0.0};
    E.sh.n_rec = 1;
    E.sh.s_init = o.s_max;
    SGM_HIP(hipMemcpyAsync(w.rec, E.sh.rec.data(), sizeof(double) * 3,
                           hipMemcpyHostToDevice, st));
  } else if (o.shifts_host != nullptr && o.n_shifts > 0) {
    E.shifts_from_host(o.shifts_host, o.n_shifts);
  }
  // r0 = b - A x0, beta0
  const int64_t np = spmv_resid(S, v64, x, b, w.r, w.P.buf, st);
  reduce_norm(w.P.buf, np, w.scal + 0, st);
  SGM_HIP(hipMemcpyAsync(hm.scal, w.scal, sizeof(double), hipMemcpyDeviceToHost,
                         st));
  wait_stream(st);
  const double beta0 = hm.scal[0];
  R.t[0] = ms_since(t0);
  auto finish = [&]() {
    if (jac) vec_scale_div(x, A.diag, n, true, st);
    wait_stream(st);
    E.flush_timing();
    R.t[7] = ms_since(t0);
  };
  if (beta0 == 0.0) {
    R.rel_true = 0.0;
    R.status = SGM_OK;
    finish();
    return;
  }
  if (!std::isfinite(beta0)) {
    R.status = SGM_ENUMERIC;
    finish();
    throw Error{SGM_ENUMERIC, "initial residual is not finite"};
  }
  SGM_HIP(hipMemcpyAsync(w.scal + 1, w.scal + 0, sizeof(double),
                         hipMemcpyDeviceToDevice, st));
  double beta = beta0;
  auto true_residual = [&]() {
    auto tc = Clock::now();
    const int64_t np2 = spmv_resid(S, v64, x, b, w.r, w.P.buf, st);
    reduce_norm(w.P.buf, np2, w.scal + 1, st);
    SGM_HIP(hipMemcpyAsync(hm.scal + 1, w.scal + 1, sizeof(double),
                           hipMemcpyDeviceToHost, st));
    wait_stream(st);
    R.t[5] += ms_since(tc);
    return hm.scal[1];
  };
  if (!f32) {
    if (!E.sh.known && !o.ritz_reuse) {
      scale_into<T>(w.r, w.scal + 1, E.Q(), 0, n, w.ld, st);
      E.cycle(w.scal + 1, w.scal + 0, o.tol, true, 1.0, nullptr);
    }
    for (;;) {
      scale_into<T>(w.r, w.scal + 1, E.Q(), 0, n, w.ld, st);
      const int k = E.cycle(w.scal + 1, w.scal + 0, o.tol, false, 1.0, nullptr);
      auto tc = Clock::now();
      if (ilu) {
        // right preconditioning: x += M^{-1} (Q y)
        SGM_HIP(hipMemsetAsync(w.ilu_z, 0, sizeof(double) * n, st));
        gemv_update<T>(E.Q().template as<const T>(), w.y, k, nullptr,
                       w.ilu_z, n, st);
        ilu_apply(*A.ilu, n, colmajor_view<const double>(w.ilu_z, w.ld),
                  w.ilu_z, w.ilu_z, st);
        axpy_f64(w.ilu_z, x, n, st);
      } else {
        gemv_update<T>(E.Q().template as<const T>(), w.y, k, nullptr, x, n,
                       st);
      }
      R.t[5] += ms_since(tc);
      R.iters += k;
      beta = true_residual();
      R.rel_true = beta / beta0;
      if (!std::isfinite(R.rel_true)) {
        finish();
        throw Error{SGM_ENUMERIC, "true residual is not finite"};
      }
      if (R.rel_true <= o.tol) {
        R.status = SGM_OK;
        break;
      }
      if (R.restarts >= o.max_restarts || k == 0) break;
      R.restarts += 1;
    }
  } else {
    // float32 inner cycles inside float64 iterative refinement
    auto tir = Clock::now();
    if (!E.sh.known && !o.ritz_reuse) {
      scale_into<T>(w.r, w.scal + 1, E.Q(), 0, n, w.ld, st);
      E.cycle(w.scal + 2, w.scal + 2, o.inner_tol, true, 1.0, nullptr);
    }
    R.rel_true = 1.0;
    while (R.outer < o.max_outer) {
      scale_into<T>(w.r, w.scal + 1, E.Q(), 0, n, w.ld, st);
      const double scale = beta / beta0;
      const int k =
          E.cycle(w.scal + 2, w.scal + 2, o.inner_tol, false, scale, nullptr);
      R.outer += 1;
      R.iters += k;
      gemv_update<T>(E.Q().template as<const T>(), w.y, k, w.scal + 1, x, n,
                     st);
      beta = true_residual();
      R.rel_true = beta / beta0;
      if (!std::isfinite(R.rel_true)) {
        finish();
        throw Error{SGM_ENUMERIC, "true residual is not finite"};
      }
      if (R.rel_true <= o.tol) {
        R.status = SGM_OK;
        break;
      }
      if (k == 0) break;
    }
    R.restarts = R.outer > 0 ? R.outer - 1 : 0;
    R.t[6] = ms_since(tir);
  }
  finish();
  R.s0 = E.sh.s0;
  R.s_init = E.sh.s_init;
  R.n_rec = E.sh.n_rec;
  R.hits = E.sh.hits;
}

}  // namespace
}  // namespace sgm

// ====================================================================== ABI
namespace {

using namespace sgm;

Handle* handle(sgm_matrix A) { return reinterpret_cast<Handle*>(A); }

#define SGM_API_BEGIN try {
#define SGM_API_END                                                        \
  }                                                                        \
  catch (const Error& e) {                                                 \
    set_error(e.msg);                                                      \
    return e.st;                                                           \
  }                                                                        \
  catch (const std::exception& e) {                                        \
    set_error(e.what());                                                   \
    return SGM_EHIP;                                                       \
  }                                                                        \
  catch (...) {                                                            \
    set_error("unknown error");                                            \
    return SGM_EHIP;                                                       \
  }

// The same for the entry points that synchronise their stream: an error
// after launches were queued waits for them before returning, so the
// caller may release the buffers they use.
#define SGM_API_END_SYNC(stream)                                           \
  }                                                                        \
  catch (const Error& e) {                                                 \
    set_error(e.msg);                                                      \
    if (e.st != SGM_EINVAL) drain(stream);                                 \
    return e.st;                                                           \
  }                                                                        \
  catch (const std::exception& e) {                                        \
    set_error(e.what());                                                   \
    drain(stream);                                                         \
    return SGM_EHIP;                                                       \
  }                                                                        \
  catch (...) {                                                            \
    set_error("unknown error");                                            \
    drain(stream);                                                         \
    return SGM_EHIP;                                                       \
  }

void validate_opts(const sgm_opts* o) {
  SGM_REQUIRE(o != nullptr, "opts is NULL");
  SGM_REQUIRE(o->s_max >= 1 && o->s_max <= 256, "s_max must be in [1, 256]");
  SGM_REQUIRE(o->restart >= 1 && o->restart <= 4096,
              "restart must be in [1, 4096]");
  SGM_REQUIRE(o->max_restarts >= 0, "max_restarts must be >= 0");
  SGM_REQUIRE(o->tol > 0.0 && std::isfinite(o->tol), "tol must be > 0");
  SGM_REQUIRE(o->precond == SGM_PRECOND_NONE ||
                  o->precond == SGM_PRECOND_JACOBI ||
                  o->precond == SGM_PRECOND_ILU0,
              "unknown preconditioner");
  if (o->precond == SGM_PRECOND_ILU0) {
    SGM_REQUIRE(o->precision == SGM_FP64,
                "the ILU(0) preconditioner runs in float64 only");
    SGM_REQUIRE(o->transpose == 0,
                "the ILU(0) preconditioner is not available for A^T solves");
  }
  SGM_REQUIRE(o->basis == SGM_BASIS_SCALED_NEWTON ||
                  o->basis == SGM_BASIS_NEWTON ||
                  o->basis == SGM_BASIS_MONOMIAL,
              "unknown basis");
  SGM_REQUIRE(o->precision == SGM_FP64 || o->precision == SGM_FP32_IR,
              "unknown precision");
  SGM_REQUIRE(o->omega >= 0.0 && o->omega_est >= 0.0,
              "omega and omega_est must be >= 0");
  if (o->precision == SGM_FP32_IR) {
    SGM_REQUIRE(o->inner_tol > 0.0 && o->inner_tol < 1.0,
                "inner_tol must be in (0, 1)");
    SGM_REQUIRE(o->max_outer >= 1, "max_outer must be >= 1");
  }
  if (o->shifts_host != nullptr)
    SGM_REQUIRE(o->n_shifts >= 1 && o->n_shifts <= 1024,
                "n_shifts must be in [1, 1024]");
  SGM_REQUIRE(o->prephase == SGM_PREPHASE_CGS2 ||
                  o->prephase == SGM_PREPHASE_MONOMIAL,
              "unknown prephase");
  SGM_REQUIRE(o->prephase_s >= 1, "prephase_s must be >= 1");
  SGM_REQUIRE(o->orth == SGM_ORTH_BCGS2 || o->orth == SGM_ORTH_BCGS2_PYTH,
              "unknown orth");
  SGM_REQUIRE(o->mpk_depth >= 1 && o->mpk_depth <= kMaxMpkTasks,
              "mpk_depth must be in [1, 4]");
}

int nshift_max(const sgm_opts& o) {
  if (o.shifts_host != nullptr) return o.n_shifts;
  return std::min(o.s_max, o.restart);
}

size_t solve_ws_bytes(const Matrix& M, const sgm_opts& o) {
  Arena a;
  Work w;
  const int64_t snnz = std::max(M.fwd.nnz_padded, M.trn.nnz_padded);
  layout(a, w, M.n, snnz, o.restart, o.s_max, nshift_max(o),
         o.precision == SGM_FP32_IR, o.precond == SGM_PRECOND_JACOBI,
         o.precond == SGM_PRECOND_ILU0);
  return a.off + 256;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// waits for the stream without throwing, and clears the sticky error
void drain(void* stream) {
  (void)hipStreamSynchronize(as_stream(stream));
  (void)hipGetLastError();
}

// Workspace of the stand-alone block orthogonalisation.
void block_layout(Arena& a, Work& w, int i, int s, int64_t n_rows) {
  w.ldw = std::max(i, 1) + s;  // room for [R2; Gram] of the Pythagorean pass
  w.lds = s;
  w.P.cap = part_cap(i, s, n_rows);
  w.P.buf = a.take<double>(w.P.cap);
  const int64_t ws = (int64_t)w.ldw * s, ss = (int64_t)s * s;
  w.W = a.take<double>(ws);
  w.R2 = a.take<double>(ws);
  w.Rtop = a.take<double>(ws);
  w.G = a.take<double>(ss);
  w.G2 = a.take<double>(ss);
  w.Z = a.take<double>(ss);
  w.Zinv = a.take<double>(ss);
  w.Zt = a.take<double>(ss);
  w.Ztinv = a.take<double>(ss);
  w.Rkk = a.take<double>(ss);
  w.pchol_scr = a.take<double>(2 * ss + 2 * s);
  w.ctrl = a.take<int>(kCtrlWords);
}

// ------------------------------------------------------- static scratch
// Device memory of sgm_block_orth_noalloc, for callers that cannot
// allocate: the small matrices of one block (W, R2, the combined R, the
// Gram matrices, both partial Cholesky factors and their inverses, the
// partial Cholesky scratch, the control words) and, in the rest, the
// partial sums of the grid reductions.  One copy per GPU, held until the
// process ends; every call on a GPU shares it, so overlapping calls on one
// GPU race.  Nothing in it needs to start at zero: every kernel writes the
// words it later reads in the same call.
constexpr size_t kStaticScratchDoubles = (size_t)3 << 20;  // 24 MiB
constexpr int kNoAllocMaxS = 64;       // block columns
constexpr int kNoAllocMaxCols = 256;   // prior + block columns (i + s)
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device
// with that device current (the array's name is only a host-side stand-in
// in host code).
double* static_scratch() {
  int dev = -1;
  SGM_HIP(hipGetDevice(&dev));
  SGM_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* ptr = nullptr;
    SGM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    SGM_REQUIRE(ptr != nullptr, "static scratch has no device address");
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[dev];
}

// block_layout in the static array: the small matrices first, then the
// partial sums in everything that is left (the reductions pick their row
// chunk counts to fit it).
void block_layout_static(Arena& a, Work& w, int i, int s) {
  w.ldw = std::max(i, 1) + s;
  w.lds = s;
  const int64_t ws = (int64_t)w.ldw * s, ss = (int64_t)s * s;
  w.W = a.take<double>(ws);
  w.R2 = a.take<double>(ws);
  w.Rtop = a.take<double>(ws);
  w.G = a.take<double>(ss);
  w.G2 = a.take<double>(ss);
  w.Z = a.take<double>(ss);
  w.Zinv = a.take<double>(ss);
  w.Zt = a.take<double>(ss);
  w.Ztinv = a.take<double>(ss);
  w.Rkk = a.take<double>(ss);
  w.pchol_scr = a.take<double>(2 * ss + 2 * s);
  w.ctrl = a.take<int>(kCtrlWords);
  a.off = (size_t)round_up((int64_t)a.off, 256);
  const int64_t left =
      ((int64_t)(kStaticScratchDoubles * sizeof(double)) - (int64_t)a.off) /
      (int64_t)sizeof(double);
  if (left < 8 * (int64_t)w.ldw * s)
    throw Error{SGM_EINVAL, "static scratch too small for this block"};
  w.P.cap = left;
  w.P.buf = a.take<double>(left);
}

// The block orthogonalisation and the read-back shared by sgm_block_orth
// and sgm_block_orth_noalloc (w laid out by the caller).
void run_block_orth(sgm_precision precision, void* Q, int64_t ldq, int32_t i,
                    int32_t s, double omega, sgm_orth orth, Work& w,
                    hipStream_t st, int32_t* p, double* R_top, double* R_kk) {
  const bool f32 = precision == SGM_FP32_IR;
  const double om = omega > 0 ? omega : default_omega(f32);
  const bool pyth = orth == SGM_ORTH_BCGS2_PYTH;
  if (f32)
    orth_block<float>(colmajor_view<float>(static_cast<float*>(Q), ldq), ldq,
                      i, s, om, w, st, true, pyth);
  else
    orth_block<double>(colmajor_view<double>(static_cast<double*>(Q), ldq),
                       ldq, i, s, om, w, st, true, pyth);
  int ctrl[C_NCTRL];
  SGM_HIP(hipMemcpyAsync(ctrl, w.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost,
                         st));
  if (R_top)
    SGM_HIP(hipMemcpy2DAsync(R_top, sizeof(double) * (size_t)i, w.Rtop,
                             sizeof(double) * (size_t)w.ldw,
                             sizeof(double) * (size_t)i, (size_t)s,
                             hipMemcpyDeviceToHost, st));
  if (R_kk)
    SGM_HIP(hipMemcpyAsync(R_kk, w.Rkk, sizeof(double) * (size_t)s * s,
                           hipMemcpyDeviceToHost, st));
  SGM_HIP(hipStreamSynchronize(st));
  *p = ctrl[C_P2];
}

void check_block_args(sgm_precision precision, int64_t n_rows, void* Q,
                      int64_t ldq, int32_t i, int32_t s, double omega,
                      sgm_orth orth, int32_t* p) {
  SGM_REQUIRE(Q != nullptr && p != nullptr, "NULL argument");
  SGM_REQUIRE(n_rows >= 1 && ldq >= n_rows && ldq % kLdAlign == 0,
              "ldq must be >= n_rows and a multiple of 64");
  SGM_REQUIRE(i >= 1 && s >= 1 && s <= 256, "need i >= 1 and 1 <= s <= 256");
  SGM_REQUIRE(precision == SGM_FP64 || precision == SGM_FP32_IR,
              "unknown precision");
  SGM_REQUIRE(omega >= 0.0, "omega must be >= 0");
  SGM_REQUIRE(orth == SGM_ORTH_BCGS2 || orth == SGM_ORTH_BCGS2_PYTH,
              "unknown orth");
}

void shifts_layout(Arena& a, Work& w, int m0) {
  w.wr = a.take<double>(m0);
  w.wi = a.take<double>(m0);
  w.ritz = a.take<double>(2 * m0);
  w.rec = a.take<double>(3 * m0);
  w.hqr_scr = a.take<double>((int64_t)m0 * m0);
  w.leja_scr = a.take<double>((int64_t)shifts_scratch_doubles(m0));
  w.info = a.take<int>(8);
}

}  // namespace

extern "C" {

sgm_status sgm_matrix_create(int64_t n, int64_t nnz, const int32_t* row_ptr,
                             const int32_t* col, const double* val,
                             void* stream, sgm_matrix* out) {
  SGM_API_BEGIN
  SGM_REQUIRE(out != nullptr, "out is NULL");
  *out = nullptr;
  SGM_REQUIRE(n >= 1 && n < ((int64_t)1 << 31) - 64, "n out of range");
  SGM_REQUIRE(nnz >= 0 && nnz < ((int64_t)1 << 31), "nnz out of range");
  SGM_REQUIRE(row_ptr != nullptr, "row_ptr is NULL");
  SGM_REQUIRE(nnz == 0 || (col != nullptr && val != nullptr),
              "col/val is NULL");
  Handle* h = new Handle();
  try {
    h->M = matrix_create(n, nnz, row_ptr, col, val, as_stream(stream));
    SGM_HIP(hipHostMalloc(&h->pinned, kPinnedBytes,
                          hipHostMallocMapped | hipHostMallocCoherent));
    h->pinned_bytes = kPinnedBytes;
    SGM_HIP(hipHostGetDevicePointer(&h->pinned_dev, h->pinned, 0));
  } catch (...) {
    if (h->M) matrix_destroy(h->M);
    delete h;
    throw;
  }
  *out = reinterpret_cast<sgm_matrix>(h);
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_matrix_update_values(sgm_matrix A, const double* val,
                                    void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr, "matrix is NULL");
  SGM_REQUIRE(val != nullptr || handle(A)->M->nnz == 0, "val is NULL");
  matrix_update_values(handle(A)->M, val, as_stream(stream));
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_matrix_destroy(sgm_matrix A) {
  SGM_API_BEGIN
  if (A == nullptr) return SGM_OK;
  Handle* h = handle(A);
  matrix_destroy(h->M);
  if (h->pinned) (void)hipHostFree(h->pinned);
  delete h;
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_matrix_ilu0(sgm_matrix A, void* stream, int32_t* levels) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr, "matrix is NULL");
  Matrix& M = *handle(A)->M;
  ilu_build(M, as_stream(stream));
  if (levels) {
    levels[0] = M.ilu->L.nlev;
    levels[1] = M.ilu->U.nlev;
  }
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_ilu0_apply(sgm_matrix A, const double* r, double* z,
                          void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && r != nullptr && z != nullptr, "NULL argument");
  const Matrix& M = *handle(A)->M;
  SGM_REQUIRE(M.ilu != nullptr && M.ilu->ok,
              "no valid ILU(0) factors: call sgm_matrix_ilu0 first");
  ilu_apply(*M.ilu, M.n, colmajor_view<const double>(r, M.n), r, z,
            as_stream(stream));
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_ilu0_factors(sgm_matrix A, double* lu, void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && lu != nullptr, "NULL argument");
  const Matrix& M = *handle(A)->M;
  SGM_REQUIRE(M.ilu != nullptr && M.ilu->ok,
              "no valid ILU(0) factors: call sgm_matrix_ilu0 first");
  SGM_HIP(hipMemcpyAsync(lu, M.ilu->fac, sizeof(double) * (size_t)M.nnz,
                         hipMemcpyDeviceToDevice, as_stream(stream)));
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_matrix_info(sgm_matrix A, int64_t* n, int64_t* nnz,
                           int64_t* sell_nnz, int32_t* index_bytes) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr, "matrix is NULL");
  const Matrix& M = *handle(A)->M;
  if (n) *n = M.n;
  if (nnz) *nnz = M.nnz;
  if (sell_nnz) *sell_nnz = M.fwd.nnz_padded;
  if (index_bytes) {
    index_bytes[0] = M.fwd.rcol ? 2 : 4;
    index_bytes[1] = M.trn.rcol ? 2 : 4;
  }
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_spmv(sgm_matrix A, int transpose, sgm_precision precision,
                    const void* x, void* y, void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && x != nullptr && y != nullptr, "NULL argument");
  SGM_REQUIRE(precision == SGM_FP64 || precision == SGM_FP32_IR,
              "unknown precision");
  const Matrix& M = *handle(A)->M;
  const Sell& S = transpose ? M.trn : M.fwd;
  if (precision == SGM_FP64)
    spmv_plain<double>(S, S.val64, static_cast<const double*>(x),
                       static_cast<double*>(y), as_stream(stream));
  else
    spmv_plain<float>(S, S.val32, static_cast<const float*>(x),
                      static_cast<float*>(y), as_stream(stream));
  return SGM_OK;
  SGM_API_END
}

void sgm_opts_default(sgm_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->s_max = 8;
  o->restart = 64;
  o->max_restarts = 100;
  o->tol = 1e-10;
  o->precond = SGM_PRECOND_NONE;
  o->basis = SGM_BASIS_SCALED_NEWTON;
  o->precision = SGM_FP64;
  o->omega = 0.0;
  o->omega_est = 0.0;
  o->use_estimator = 1;
  o->transpose = 0;
  o->inner_tol = 1e-6;
  o->max_outer = 200;
  o->ritz_reuse = 1;
  o->shifts_host = nullptr;
  o->n_shifts = 0;
  o->prephase = SGM_PREPHASE_CGS2;
  o->prephase_s = 8;
  o->orth = SGM_ORTH_BCGS2;
  o->mpk_depth = 1;
}

sgm_status sgm_workspace_size(sgm_matrix A, const sgm_opts* o,
                              size_t* bytes) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && bytes != nullptr, "NULL argument");
  validate_opts(o);
  *bytes = solve_ws_bytes(*handle(A)->M, *o);
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_solve(sgm_matrix A, const double* b, const double* x0,
                     double* x, const sgm_opts* o, void* ws, size_t ws_bytes,
                     void* stream, double* res_hist, int32_t res_cap,
                     int32_t* s_hist, int32_t s_cap, sgm_info* info) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr, "matrix is NULL");
  SGM_REQUIRE(b != nullptr && x != nullptr, "b or x is NULL");
  validate_opts(o);
  SGM_REQUIRE(res_cap >= 0 && s_cap >= 0, "negative history capacity");
  Handle* h = handle(A);
  const size_t need = solve_ws_bytes(*h->M, *o);
  SGM_REQUIRE(ws != nullptr && ws_bytes >= need,
              "workspace too small: need " + std::to_string(need) + " bytes");
  SGM_REQUIRE(o->s_max + 1 <= (int)((kPinnedBytes - 256) / sizeof(double)),
              "s_max too large");
  Arena a;
  a.base = reinterpret_cast<char*>(
      round_up(reinterpret_cast<int64_t>(ws), 256));
  Work w;
  const int64_t snnz = std::max(h->M->fwd.nnz_padded, h->M->trn.nnz_padded);
  layout(a, w, h->M->n, snnz, o->restart, o->s_max, nshift_max(*o),
         o->precision == SGM_FP32_IR, o->precond == SGM_PRECOND_JACOBI,
         o->precond == SGM_PRECOND_ILU0);
  Result R;
  sgm_status st = SGM_OK;
  std::string err;
  try {
    if (o->precision == SGM_FP64)
      run_solve<double>(h, b, x0, x, *o, w, as_stream(stream), R);
    else
      run_solve<float>(h, b, x0, x, *o, w, as_stream(stream), R);
    st = R.status;
  } catch (const Error& e) {
    st = e.st;
    err = e.msg;
    // launches queued behind the failed step (matrix powers steps queued
    // ahead, gated off by the tail) still read the workspace: let them
    // finish before the caller may release it
    drain(stream);
  }
  if (res_hist)
    for (int32_t i = 0; i < res_cap && i < (int32_t)R.res_hist.size(); ++i)
      res_hist[i] = R.res_hist[i];
  if (s_hist)
    for (int32_t i = 0; i < s_cap && i < (int32_t)R.s_hist.size(); ++i)
      s_hist[i] = R.s_hist[i];
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->iters = R.iters;
    info->restarts = R.restarts;
    info->outer_iters = o->precision == SGM_FP32_IR ? R.outer : 0;
    info->s0_est = R.s0;
    info->s_init = R.s_init;
    info->n_hist = (int32_t)R.res_hist.size();
    info->n_blocks = (int32_t)R.s_hist.size();
    info->n_shifts = R.n_rec;
    info->gamma_guard_hits = R.hits;
    info->rel_res_true = R.rel_true;
    info->rel_res_est = R.rel_est;
    for (int i = 0; i < 8; ++i) info->t_phase_ms[i] = R.t[i];
    info->n_spmv = R.n_spmv;
    info->t_spmv_ms = R.t_spmv;
    info->mpk_depth = R.mpk_depth;
    info->mpk_slab_rows = R.mpk_slab_rows;
  }
  if (st < 0) set_error(err);
  return st;
  SGM_API_END_SYNC(stream)
}

sgm_status sgm_grad_vals(sgm_matrix A, const double* lambda, const double* x,
                         double* grad_val, void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && lambda != nullptr && x != nullptr &&
                  grad_val != nullptr,
              "NULL argument");
  grad_vals(*handle(A)->M, lambda, x, grad_val, as_stream(stream));
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_mpk(sgm_matrix A, int transpose, sgm_precision precision,
                   void* Q, int64_t ldq, int32_t c, int32_t s,
                   const double* records, int32_t n_rec, void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && Q != nullptr && records != nullptr,
              "NULL argument");
  const Matrix& M = *handle(A)->M;
  SGM_REQUIRE(ldq >= M.n && ldq % kLdAlign == 0,
              "ldq must be >= n and a multiple of 64");
  SGM_REQUIRE(c >= 0 && s >= 0 && n_rec >= 1, "bad c/s/n_rec");
  SGM_REQUIRE(precision == SGM_FP64 || precision == SGM_FP32_IR,
              "unknown precision");
  const Sell& S = transpose ? M.trn : M.fwd;
  hipStream_t st = as_stream(stream);
  for (int j = 0; j < s; ++j) {
    const int q = j % n_rec;
    const int jprev = j >= 1 ? c + j - 1 : -1;
    if (precision == SGM_FP64)
      spmv_mpk<double>(S, S.val64,
                       colmajor_view<double>(static_cast<double*>(Q), ldq),
                       c + j, jprev, c + j + 1, records, q, st);
    else
      spmv_mpk<float>(S, S.val32,
                      colmajor_view<float>(static_cast<float*>(Q), ldq),
                      c + j, jprev, c + j + 1, records, q, st);
  }
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_mpk_norms(sgm_matrix A, int transpose, sgm_precision precision,
                         void* Q, int64_t ldq, int32_t c, int32_t s,
                         const double* records, int32_t n_rec, double* norms2,
                         double* work, int64_t work_len, void* stream) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && Q != nullptr && records != nullptr,
              "NULL argument");
  const Matrix& M = *handle(A)->M;
  SGM_REQUIRE(ldq >= M.n && ldq % kLdAlign == 0,
              "ldq must be >= n and a multiple of 64");
  SGM_REQUIRE(c >= 0 && s >= 0 && n_rec >= 1, "bad c/s/n_rec");
  SGM_REQUIRE(precision == SGM_FP64 || precision == SGM_FP32_IR,
              "unknown precision");
  const Sell& S = transpose ? M.trn : M.fwd;
  SGM_REQUIRE(s == 0 || (norms2 != nullptr && work != nullptr),
              "NULL norms2 or work");
  SGM_REQUIRE(s == 0 || work_len >= resid_partials(S),
              "work must hold ceil(n / 256) doubles");
  hipStream_t st = as_stream(stream);
  for (int j = 0; j < s; ++j) {
    const int q = j % n_rec;
    const int jprev = j >= 1 ? c + j - 1 : -1;
    if (precision == SGM_FP64)
      spmv_mpk_norm<double>(
          S, S.val64, colmajor_view<double>(static_cast<double*>(Q), ldq),
          c + j, jprev, c + j + 1, records, q, work, norms2 + j, st);
    else
      spmv_mpk_norm<float>(
          S, S.val32, colmajor_view<float>(static_cast<float*>(Q), ldq),
          c + j, jprev, c + j + 1, records, q, work, norms2 + j, st);
  }
  return SGM_OK;
  SGM_API_END
}

sgm_status sgm_mpk_fused(sgm_matrix A, int transpose, sgm_precision precision,
                         void* Q, int64_t ldq, int32_t c, int32_t s,
                         const double* records, int32_t n_rec, int32_t depth,
                         void* stream, int64_t* slab_rows) {
  SGM_API_BEGIN
  SGM_REQUIRE(A != nullptr && Q != nullptr && records != nullptr,
              "NULL argument");
  const Matrix& M = *handle(A)->M;
  SGM_REQUIRE(ldq >= M.n && ldq % kLdAlign == 0,
              "ldq must be >= n and a multiple of 64");
  SGM_REQUIRE(c >= 0 && s >= 0 && n_rec >= 1, "bad c/s/n_rec");
  SGM_REQUIRE(depth >= 1 && depth <= kMaxMpkTasks, "depth must be in [1, 4]");
  SGM_REQUIRE(precision == SGM_FP64 || precision == SGM_FP32_IR,
              "unknown precision");
  const Sell& S = transpose ? M.trn : M.fwd;
  hipStream_t st = as_stream(stream);
  std::vector<MpkStep> steps(s > 0 ? s : 1);
  for (int j = 0; j < s; ++j)
    steps[j] = MpkStep{c + j, j >= 1 ? c + j - 1 : -1, c + j + 1, j % n_rec};
  const bool f32 = precision == SGM_FP32_IR;
  const MpkPlan plan = mpk_plan(S, M.bandwidth, depth, f32 ? 4 : 8);
  if (slab_rows) *slab_rows = plan.depth > 1 ? plan.slab_slices * kSlice : 0;
  if (f32)
    spmv_mpk_steps<float>(S, S.val32,
                          colmajor_view<float>(static_cast<float*>(Q), ldq),
                          steps.data(), s, records, plan, st);
  else
    spmv_mpk_steps<double>(S, S.val64,
                           colmajor_view<double>(static_cast<double*>(Q), ldq),
                           steps.data(), s, records, plan, st);
  return SGM_OK;
  SGM_API_END
}

size_t sgm_block_ws_size(int64_t n_rows, int32_t i, int32_t s) {
  if (i < 1 || s < 1) return 0;
  Arena a;
  Work w;
  block_layout(a, w, i, s, n_rows);
  return a.off + 256;
}

sgm_status sgm_block_orth(sgm_precision precision, int64_t n_rows, void* Q,
                          int64_t ldq, int32_t i, int32_t s, double omega,
                          sgm_orth orth, void* ws, size_t ws_bytes,
                          void* stream, int32_t* p, double* R_top,
                          double* R_kk) {
  SGM_API_BEGIN
  check_block_args(precision, n_rows, Q, ldq, i, s, omega, orth, p);
  const size_t need = sgm_block_ws_size(n_rows, i, s);
  SGM_REQUIRE(ws != nullptr && ws_bytes >= need, "workspace too small");
  Arena a;
  a.base = reinterpret_cast<char*>(
      round_up(reinterpret_cast<int64_t>(ws), 256));
  Work w;
  block_layout(a, w, i, s, n_rows);
  run_block_orth(precision, Q, ldq, i, s, omega, orth, w, as_stream(stream),
                 p, R_top, R_kk);
  return SGM_OK;
  SGM_API_END_SYNC(stream)
}

sgm_status sgm_block_orth_noalloc(sgm_precision precision, int64_t n_rows,
                                  void* Q, int64_t ldq, int32_t i, int32_t s,
                                  double omega, sgm_orth orth, void* stream,
                                  int32_t* p, double* R_top, double* R_kk) {
  SGM_API_BEGIN
  check_block_args(precision, n_rows, Q, ldq, i, s, omega, orth, p);
  SGM_REQUIRE(s <= kNoAllocMaxS && i + s <= kNoAllocMaxCols,
              "sgm_block_orth_noalloc: needs s <= 64 and i + s <= 256 (its "
              "static scratch holds 24 MiB); use sgm_block_orth for larger "
              "blocks");
  Arena a;
  a.base = reinterpret_cast<char*>(static_scratch());
  Work w;
  block_layout_static(a, w, i, s);
  run_block_orth(precision, Q, ldq, i, s, omega, orth, w, as_stream(stream),
                 p, R_top, R_kk);
  return SGM_OK;
  SGM_API_END_SYNC(stream)
}

size_t sgm_shifts_ws_size(int32_t m0) {
  if (m0 < 1) return 0;
  Arena a;
  Work w;
  shifts_layout(a, w, m0);
  return a.off + 256;
}

sgm_status sgm_shifts(const double* H, int32_t ldh, int32_t m0,
                      sgm_basis basis, double eps, double omega_est,
                      void* ws, size_t ws_bytes, void* stream,
                      double* ritz_re, double* ritz_im, double* records,
                      int32_t* s0, int32_t* guard_hits) {
  SGM_API_BEGIN
  SGM_REQUIRE(H != nullptr, "H is NULL");
  SGM_REQUIRE(m0 >= 1 && m0 <= 1024 && ldh >= m0, "need 1 <= m0 <= 1024, ldh >= m0");
  SGM_REQUIRE(eps > 0.0 && eps < 1.0, "eps must be in (0, 1)");
  SGM_REQUIRE(omega_est >= 0.0, "omega_est must be >= 0");
  SGM_REQUIRE(basis == SGM_BASIS_SCALED_NEWTON || basis == SGM_BASIS_NEWTON ||
                  basis == SGM_BASIS_MONOMIAL,
              "unknown basis");
  const size_t need = sgm_shifts_ws_size(m0);
  SGM_REQUIRE(ws != nullptr && ws_bytes >= need, "workspace too small");
  Arena a;
  a.base = reinterpret_cast<char*>(
      round_up(reinterpret_cast<int64_t>(ws), 256));
  Work w;
  shifts_layout(a, w, m0);
  hipStream_t st = as_stream(stream);
  hqr_eigen(H, ldh, m0, w.wr, w.wi, w.hqr_scr, w.info, st);
  leja_records(w.wr, w.wi, m0, (int)basis, eps,
               basis == SGM_BASIS_SCALED_NEWTON ? omega_est : 0.0, w.ritz,
               w.rec, w.info + 1, w.leja_scr, st);
  int info[4];
  std::vector<double> ritz(2 * (size_t)m0), rec(3 * (size_t)m0);
  SGM_HIP(hipMemcpyAsync(info, w.info, sizeof(info), hipMemcpyDeviceToHost,
                         st));
  SGM_HIP(hipMemcpyAsync(ritz.data(), w.ritz, sizeof(double) * ritz.size(),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipMemcpyAsync(rec.data(), w.rec, sizeof(double) * rec.size(),
                         hipMemcpyDeviceToHost, st));
  SGM_HIP(hipStreamSynchronize(st));
  if (ritz_re)
    for (int k = 0; k < m0; ++k) ritz_re[k] = ritz[2 * k];
  if (ritz_im)
    for (int k = 0; k < m0; ++k) ritz_im[k] = ritz[2 * k + 1];
  if (records) std::memcpy(records, rec.data(), sizeof(double) * rec.size());
  if (s0) *s0 = info[1];
  if (guard_hits) *guard_hits = info[2];
  if (info[0] != 0 || info[3] != 0)
    throw Error{SGM_ENUMERIC, "QR iteration failed or non-finite Ritz values"};
  return SGM_OK;
  SGM_API_END_SYNC(stream)
}

const char* sgm_status_string(sgm_status s) {
  switch (s) {
    case SGM_OK: return "ok";
    case SGM_NOT_CONVERGED: return "not converged";
    case SGM_EINVAL: return "invalid argument";
    case SGM_EHIP: return "HIP error";
    case SGM_ENOMEM: return "out of device memory";
    case SGM_ENUMERIC: return "numerical breakdown (NaN/Inf)";
  }
  return "unknown status";
}

const char* sgm_last_error(void) { return last_error(); }

int sgm_device_ok(void) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return 0;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, 0) != hipSuccess) return 0;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

}  // extern "C"
