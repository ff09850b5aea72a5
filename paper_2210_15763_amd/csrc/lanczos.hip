// Host driver and C ABI of libbbl.so: non-restarted block Lanczos (Methods,
// "Block Lanczos algorithm") with a random or bootstrapped pivot block.
//
// One iteration J (0-based; block V_{J+1} of the paper is basis slot J):
//   W   = H V_J                                   (SpMM, basis precision)
//   A_J = sym(V_J^T W)                            (MFMA gram)
//   W'  = W - V_J A_J - V_{J-1} B_{J-1}^T         (MFMA update, FP64 out)
//   W' -= V_{0:J} (V_{0:J}^T W'), twice           (full reorthogonalisation)
//   W'  = V_{J+1} B_J                             (spectral factor of the
//         overlap with deflation, then a Cholesky polish; V_{J+1} stored in
//         basis precision, B_J upper triangular)
//   every few blocks: lowest Ritz pairs of the band matrix, residual
//   estimates ||B_J s_last||; when all pass, Ritz vectors and the explicit
//   FP64 residual decide convergence.
// A block first runs a fast path: one Gram-Schmidt sweep and a Cholesky QR.
// Whether it needed the second sweep (the DGKS norm test) or the spectral
// factor with deflation is recorded on the device and read by the host two
// blocks later (the queue keeps two blocks ahead of the host); such a block
// (rare: none on the benchmark matrices) is then redone on the full path,
// which decides both branches on the device, and the blocks queued after it
// are discarded.
// Every step runs in HIP kernels.  The recurrence runs on the caller's stream;
// the band eigensolve of a check runs on a second stream of the solver,
// concurrently with the recurrence, and its result is read by the host once
// the block it ends with has been verified (two blocks later, always at the
// same point of the sequence, so the run is deterministic).  The host only
// sequences launches and reads 2k+3 numbers per check and 3 per block.
#include <chrono>
#include <deque>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bandeig.h"
#include "common.h"
#include "driver.h"
#include "pivot.h"
#include "small.h"

namespace bbl {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

constexpr int kMaxPartialRows = 4096;   // residual / column-statistics partials
constexpr uint32_t kTagDeflation = 7;
constexpr int kHn2Slot = 200;          // dres slot: max |A_jj| seen so far (<= ||H||)
constexpr int kHn2Snap = 202;          // dres slots 202..205: kHn2Slot at the start of block J (J % 4)
constexpr int kBreakSnap = 128;        // ints 128..131: the breakdown flag at the start of block J (J % 4)
// chk (256 doubles): [0, 2k] a check's Ritz values, estimates and ||T||_est
// (k <= 32: up to index 64); [128, 194) a restart's eigensolve results;
// kChkFlag: the breakdown flag as of the check's launch (one int)
constexpr int kChkFlag = 240;

size_t dsize(int dt) { return dt == BBL_F32 ? 4 : 8; }


struct Layout {
  size_t basis, W, Wp, X, partial, C, band, Bstore, mats, ints, dres, chk, S, eig, norm, Sp, total;
  size_t partial_doubles;
  BandEigLayout el;
};

// keep > 0: thick restart keeping `keep` Ritz vectors -- keep / b more basis
// slots (the rotated Ritz vectors are formed there), eigenpairs and
// coefficients for keep vectors.
Layout make_layout(int64_t n, int b, int k, int m_max, int bdt, int keep = 0) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t sx = dsize(bdt);
  const int64_t Mmax = (int64_t)(m_max + 1) * b;
  const int nyw = std::max(b, k);
  const int kS = std::max(k, keep);  // eigenpairs of a band solve
  L.basis = take((size_t)(m_max + 1 + keep / b) * n * b * sx);
  L.W = take((size_t)n * b * sx);
  L.Wp = take((size_t)n * b * 8);
  L.X = take((size_t)n * k * 8);
  L.partial_doubles =
      std::max(gram_partial_doubles(Mmax, nyw), (size_t)kMaxPartialRows * nyw * 9 / 8 + 4096);
  L.partial = take(L.partial_doubles * 8);
  L.C = take((size_t)Mmax * nyw * 8);
  L.band = take((size_t)(Mmax + b) * (b + 1) * 8);
  L.Bstore = take((size_t)(m_max + 1) * b * b * 8);
  L.mats = take((size_t)16 * kMaxBlock * kMaxBlock * 8);
  L.ints = take(256 * sizeof(int));
  L.dres = take(256 * 8);
  L.chk = take(256 * 8);
  L.S = take((size_t)m_max * b * kS * 8);
  L.el = band_eig_layout(m_max * b, b, kS);
  L.eig = take(L.el.bytes);
  L.norm = take(normalize_scratch_bytes(k, kMaxPartialRows));
  L.Sp = take(keep > 0 ? ((size_t)m_max * b * keep + kMaxBlock * kMaxBlock) * 8 : 0);
  L.total = off + 256;
  return L;
}


// The second stream of the overlapped convergence checks, its events, a
// pinned host buffer for the check results and the timing events of one
// solve.  Non-blocking, so that it never synchronises implicitly with a legacy
// default stream of the caller.  The pinned buffer also receives, per block of
// the fast path, its rare-branch flags (slot J % kRing: ints flag2, -,
// chol_fail at kIterFlags + 4 (J % kRing)) and `fev[J % kRing]` marks their
// arrival.  The host reads a block's flags kLag blocks later, so kRing > kLag
// slots are in use at a time.
//
// These are created once and kept for the life of the process in a per-device
// pool (a solve takes one set and gives it back when it returns), so a solve
// -- and every truncated solve of a pivot -- creates no stream, event or
// pinned buffer of its own.
constexpr int kLag = 2, kRing = 4;
// A convergence check is read this many blocks after the block it ends with
// (and once that block is verified).  Problems of fewer than kShortRows rows
// (blocks of about 0.1-0.3 ms) read it later than kLag: the band eigensolve
// takes about 0.7 ms whatever n, and a host that waited for it sooner would
// leave the main stream idle (n = 20,000, b = 8, 91-94 blocks: 21.0 ms with
// kLag, 18.6 ms with 4).  The lag is a function of the problem, not of
// timing, so the check schedule and the results stay deterministic.
#ifndef BBL_CHECK_LAG_SHORT
#define BBL_CHECK_LAG_SHORT 4
#endif
constexpr int kCheckLagShort = BBL_CHECK_LAG_SHORT;
constexpr int64_t kShortRows = int64_t(1) << 19;
constexpr int kIterFlags = 2 * (2 * kMaxBlock + 8);  // int offset in the pinned buffer

// Phase boundaries recorded per block instance when phase timing is on:
// [0] before the SpMM, [1] after it, [2] after the three-term step, [3] after
// the reorthogonalisation, [4] after the block QR.
constexpr int kPhaseEv = 5, kTimeRing = 8;

struct CheckStream {
  int device = -1;
  hipStream_t cs = nullptr;
  hipEvent_t ready = nullptr, done = nullptr, fev[kRing] = {};
  hipEvent_t tev[kTimeRing][kPhaseEv] = {};  // timing events, per block instance
  hipEvent_t eig0 = nullptr, eig1 = nullptr;  // around a check's band eigensolve
  hipEvent_t rs0 = nullptr, rs1 = nullptr;    // around a thick restart
  double *host = nullptr;
  static constexpr int kHostDoubles = 2 * kMaxBlock + 16;
  void create() {
    BBL_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    BBL_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    BBL_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    for (auto &e : fev) BBL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &row : tev)
      for (auto &e : row) BBL_HIP(hipEventCreate(&e));
    BBL_HIP(hipEventCreate(&eig0));
    BBL_HIP(hipEventCreate(&eig1));
    BBL_HIP(hipEventCreate(&rs0));
    BBL_HIP(hipEventCreate(&rs1));
    BBL_HIP(hipHostMalloc(reinterpret_cast<void **>(&host), kHostDoubles * sizeof(double),
                          hipHostMallocDefault));
  }
  int *iter_flags(int J) { return reinterpret_cast<int *>(host) + kIterFlags + 4 * (J % kRing); }
};

std::mutex g_pool_mu;
std::vector<CheckStream *> g_pool;  // idle sets, any device; never freed

CheckStream *acquire_check_stream() {
  int dev = 0;
  BBL_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t i = 0; i < g_pool.size(); ++i)
      if (g_pool[i]->device == dev) {
        CheckStream *c = g_pool[i];
        g_pool.erase(g_pool.begin() + i);
        return c;
      }
  }
  CheckStream *c = new CheckStream();
  c->device = dev;
  try {
    c->create();
  } catch (...) {
    delete c;  // (its partially created handles are left to the process exit)
    throw;
  }
  return c;
}

void release_check_stream(CheckStream *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->cs);  // nothing of this solve may still run on it
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pool.push_back(c);
}

// Holds a pooled set for the duration of one solve.
struct CheckStreamLease {
  CheckStream *c;
  hipStream_t s;
  explicit CheckStreamLease(hipStream_t s_) : c(acquire_check_stream()), s(s_) {}
  ~CheckStreamLease() {
    (void)hipStreamSynchronize(s);  // its flag copies target the pinned buffer
    release_check_stream(c);
  }
  CheckStream &operator*() { return *c; }
  CheckStreamLease(const CheckStreamLease &) = delete;
  CheckStreamLease &operator=(const CheckStreamLease &) = delete;
};

// Device time per phase of the recurrence (HIP events on the solver's stream
// around the SpMM, the three-term step, the reorthogonalisation and the block
// QR of every block instance, redone and discarded ones included), read back
// kTimeRing instances later, when the event set is reused, and at the end.
struct PhaseTimer {
  bool spmm_on = false, all_on = false;
  CheckStream *cq = nullptr;
  int64_t inst = 0, harvested = 0;
  double ms[4] = {0, 0, 0, 0};  // spmm, three-term, reorth, qr
  int spmm_count = 0;
  void harvest_one(int64_t i) {
    hipEvent_t *e = cq->tev[i % kTimeRing];
    const int last = all_on ? kPhaseEv - 1 : 1;
    BBL_HIP(hipEventSynchronize(e[last]));
    for (int p = 0; p < last; ++p) {
      float t = 0.f;
      BBL_HIP(hipEventElapsedTime(&t, e[p], e[p + 1]));
      ms[p] += t;
    }
    ++spmm_count;
  }
  // Starts block instance i; returns its event set (nullptr when timing is off).
  hipEvent_t *begin() {
    if (!spmm_on) return nullptr;
    if (inst - harvested >= kTimeRing) harvest_one(harvested++);
    return cq->tev[inst++ % kTimeRing];
  }
  void mark(hipEvent_t *e, int p, hipStream_t s) {
    if (e && (all_on || p <= 1)) BBL_HIP(hipEventRecord(e[p], s));
  }
  void finish() {
    while (harvested < inst) harvest_one(harvested++);
  }
};

struct Solver {
  const bbl_csr &H;
  int64_t n;
  int b, k;
  double tol;
  Opts o;
  hipStream_t s;
  Layout L;
  char *ws;
  int xd;  // basis dtype
  size_t sx;
  // regions
  char *basis;
  void *W;
  double *Wp, *X, *partial, *C, *band, *Bstore, *S, *dres, *chk;
  double *Araw, *C3, *O, *C0, *QB, *RB, *O2, *Rinv, *G0, *G1;
  int *ints;
  int *mask, *flag, *breakdown, *ndefl, *flag2, *n_second, *chol_fail;
  void *eigws, *normws;
  double *Sp = nullptr, *Qr = nullptr;  // thick restart: coefficients, rotation
  int qr_calls = 0;

  Solver(const bbl_csr &H_, int b_, int k_, double tol_, const Opts &o_, void *ws_, size_t bytes,
         hipStream_t s_)
      : H(H_), n(H_.n), b(b_), k(k_), tol(tol_), o(o_), s(s_) {
    xd = o.basis_dtype;
    sx = dsize(xd);
    L = make_layout(n, b, k, o.m_max, xd, o.restart_keep);
    if (bytes < L.total) throw Error{BBL_E_NOMEM, "workspace too small"};
    ws = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws_), 256));
    basis = ws + L.basis;
    W = ws + L.W;
    Wp = reinterpret_cast<double *>(ws + L.Wp);
    X = reinterpret_cast<double *>(ws + L.X);
    partial = reinterpret_cast<double *>(ws + L.partial);
    C = reinterpret_cast<double *>(ws + L.C);
    band = reinterpret_cast<double *>(ws + L.band);
    Bstore = reinterpret_cast<double *>(ws + L.Bstore);
    S = reinterpret_cast<double *>(ws + L.S);
    dres = reinterpret_cast<double *>(ws + L.dres);
    chk = reinterpret_cast<double *>(ws + L.chk);
    double *m = reinterpret_cast<double *>(ws + L.mats);
    const int sq = kMaxBlock * kMaxBlock;
    Araw = m;
    C3 = m + 1 * sq;  // 2 squares
    O = m + 3 * sq;
    C0 = m + 4 * sq;
    QB = m + 5 * sq;
    RB = m + 6 * sq;
    O2 = m + 7 * sq;
    Rinv = m + 8 * sq;
    G0 = m + 9 * sq;
    G1 = m + 10 * sq;
    ints = reinterpret_cast<int *>(ws + L.ints);
    mask = ints;
    flag = ints + 64;
    breakdown = ints + 65;
    ndefl = ints + 66;
    flag2 = ints + 67;
    n_second = ints + 68;
    chol_fail = ints + 69;
    eigws = ws + L.eig;
    normws = ws + L.norm;
    Sp = reinterpret_cast<double *>(ws + L.Sp);
    Qr = Sp + (size_t)o.m_max * b * o.restart_keep;
  }

  char *slot(int J) const { return basis + (size_t)J * n * b * sx; }
  int64_t slot_stride() const { return n * b; }

  int max_partials(int M, int ny) const {
    return gram_max_partials(L.partial_doubles, M, ny);
  }

  // C (M x ny) = X^T Y with X = nblk basis-type blocks
  void gram(const void *Xp, int xdt, int bx, int nblk, int64_t xstride, const void *Y, int ydt,
            int ny, double *out, const int *when = nullptr) {
    const int M = nblk * bx;
    const int P = launch_gram_when(n, Xp, xdt, bx, nblk, xstride, Y, ydt, ny, partial,
                                   max_partials(M, ny), when, s);
    launch_reduce_when(partial, P, M, ny, out, when, s);
  }

  // Yout = beta Yin + alpha X C (b x b C) and G = Yout^T Yout, the latter
  // from the update's own partials where it can produce them.
  void update_gram(const void *Xp, int xdt, int nblk, int64_t xstride, const double *Cm,
                   double alpha, const void *Yin, int yindt, double beta, double *Yout, double *G,
                   const int *when) {
    const int P = launch_update_gram_when(n, Xp, xdt, b, nblk, xstride, Cm, b, alpha, Yin, yindt,
                                          beta, Yout, BBL_F64, partial, L.partial_doubles, when, s);
    if (P > 0) launch_reduce_when(partial, P, b, b, G, when, s);
    else gram(Yout, BBL_F64, b, 1, 0, Yout, BBL_F64, b, G, when);
  }

  // Full reorthogonalisation of W' (whose Gram G0 is known) against the
  // stored blocks, leaving G1 = W'^T W' of the result: one classical
  // Gram-Schmidt sweep, and a second one decided on the device when the
  // first removed a large part of some column (norm ratio below 1/sqrt(2)).
  void reorth_recurrence(int nb, double *Y) {
    gram(basis, xd, b, nb, slot_stride(), Y, BBL_F64, b, C);
    update_gram(basis, xd, nb, slot_stride(), C, -1.0, Y, BBL_F64, 1.0, Y, G1, nullptr);
    launch_reorth_check(G0, G1, b, 0.5, nullptr, flag2, n_second, s);
    gram(basis, xd, b, nb, slot_stride(), Y, BBL_F64, b, C, flag2);
    update_gram(basis, xd, nb, slot_stride(), C, -1.0, Y, BBL_F64, 1.0, Y, G1, flag2);
  }

  // One classical Gram-Schmidt sweep: W' -= V_{0:nb-1} (V^T W').
  void cgs_pass(int nb, double *Y, const int *when) {
    gram(basis, xd, b, nb, slot_stride(), Y, BBL_F64, b, C, when);
    launch_update_when(n, basis, xd, b, nb, slot_stride(), C, b, -1.0, Y, BBL_F64, 1.0, Y,
                       BBL_F64, when, s);
  }

  // Two unconditional sweeps (fresh random directions after a deflation).
  void reorth_twice(int nb, double *Y, const int *when) {
    cgs_pass(nb, Y, when);
    cgs_pass(nb, Y, when);
  }

  // Block QR of Wp into basis slot `dest`; Bout = B (upper triangular).
  // Oknown: Wp^T Wp if the caller has it (else it is formed here).
  void block_qr(int nbasis, int dest, double *Bout, const double *hnorm_dev,
                const double *Oknown = nullptr) {
    if (!Oknown) gram(Wp, BBL_F64, b, 1, 0, Wp, BBL_F64, b, O);
    const double *Ov = Oknown ? Oknown : O;
    launch_chol_try(Ov, b, o.tau, hnorm_dev, dres + kHn2Slot, C0, QB, RB, mask, flag, chol_fail,
                    s);
    launch_svqb_prepare(Ov, b, o.tau, hnorm_dev, dres + kHn2Slot, C0, QB, RB, mask, flag, ndefl,
                        chol_fail, s);
    // Wp C0 and its Gram O2 (final unless a column was deflated)
    update_gram(Wp, BBL_F64, 1, 0, C0, 1.0, nullptr, BBL_F64, 0.0, Wp, O2, nullptr);
    // deflated columns: fresh random directions, orthogonal to the basis
    const uint64_t key = (o.seed ^ 0x9E3779B97F4A7C15ull) + 0x5DEECE66Dull * (uint64_t)(qr_calls + 1);
    launch_gauss(n, b, b, 0, key, kTagDeflation, Wp, mask, flag, s);
    if (nbasis > 0) reorth_twice(nbasis, Wp, flag);
    update_gram(Wp, BBL_F64, 1, 0, QB, 1.0, nullptr, BBL_F64, 0.0, Wp, O2, flag);
    launch_chol_finish(O2, b, RB, Rinv, Bout, breakdown, s);
    launch_update(n, Wp, BBL_F64, b, 1, 0, Rinv, b, 1.0, nullptr, BBL_F64, 0.0, slot(dest), xd,
                  s);
    ++qr_calls;
  }

  struct Result {
    bool converged = false;
    int iters = 0, built = 0, spmm_calls = 0, checks = 0, spmm_timed = 0, restarts = 0;
    int done_blocks = 0;  // block iterations of the cycles before the current one
    int cycle_q = 0;      // blocks of kept Ritz vectors that open the current cycle
    double hnorm = 0.0, spmm_ms = 0.0, threeterm_ms = 0.0, reorth_ms = 0.0, qr_ms = 0.0,
           eig_ms = 0.0, restart_ms = 0.0;
    std::vector<double> theta, resid;
  };

  // When to solve the band matrix next.  A fixed interval if the caller asked
  // for one; otherwise the decay of the largest residual estimate between the
  // last two checks is extrapolated to the tolerance and half of the predicted
  // distance is skipped (at least 1, at most 8 blocks), so the eigensolve runs
  // a few dozen times per solve instead of every block.
  int next_check_after(int nblk, double rho_max, double target) {
    if (o.check_every > 0) return nblk + o.check_every;
    const double lr = std::log(std::max(rho_max, 1e-300));
    int step = 2;
    if (have_prev_ && nblk > prev_nblk_) {
      const double rate = (lr - prev_log_rho_) / (double)(nblk - prev_nblk_);
      if (rate < -1e-6) {
        const double togo = (std::log(std::max(target, 1e-300)) - lr) / rate;
        step = (int)std::floor(0.5 * togo);
      }
    }
    step = std::max(1, std::min(8, step));
    have_prev_ = true;
    prev_nblk_ = nblk;
    prev_log_rho_ = lr;
    return nblk + step;
  }
  bool have_prev_ = false;
  int prev_nblk_ = 0;
  double prev_log_rho_ = 0.0;

  // Ritz vectors of the last (completed) check into Xout (n x k), normalised;
  // returns their explicit residual norms ||H x - theta x|| with the check's
  // Ritz values theta = chk[0..kk).
  std::vector<double> ritz_and_residual(int nblk, int kk, double *Xout) {
    launch_update(n, basis, xd, b, nblk, slot_stride(), S, kk, 1.0, nullptr, BBL_F64, 0.0, Xout,
                  BBL_F64, s);
    launch_normalize_columns(n, kk, Xout, reinterpret_cast<double *>(normws), kMaxPartialRows, s);
    const int P = launch_residual_spmm(H, Xout, kk, chk, partial, kMaxPartialRows, s);
    double *r2 = dres + 128;
    launch_reduce(partial, P, 1, kk, r2, s);
    std::vector<double> h(kk);
    BBL_HIP(hipMemcpyAsync(h.data(), r2, kk * sizeof(double), hipMemcpyDeviceToHost, s));
    BBL_HIP(hipStreamSynchronize(s));
    for (auto &v : h) v = std::sqrt(std::max(v, 0.0));
    return h;
  }

  // A check of the first nblk blocks: the band eigensolve on the check
  // stream once the recurrence has produced B_{nblk-1}.  chk[0..2kk] receives
  // the Ritz values, residual estimates and ||T||_est, chk[kChkFlag] (as int)
  // the QR breakdown flag as of this point; both are copied to pinned memory.
  // A check due at the end of a block is armed there and launched right
  // after the next block's SpMM is queued, so that it runs beside that block's
  // tall-skinny products instead of holding compute units the SpMM needs (a
  // planned-SpMM workgroup takes a whole CU's LDS).  It reads only band rows
  // of blocks that are complete.
  int armed_nblk_ = 0, armed_kk_ = 0;
  void arm_check(int nblk, int kk) {
    armed_nblk_ = nblk;
    armed_kk_ = kk;
  }
  void fire_armed(CheckStream &cq) {
    if (!armed_nblk_) return;
    const int nb = armed_nblk_, kk = armed_kk_;
    armed_nblk_ = 0;
    launch_check(cq, nb, kk);
  }

  void launch_check(CheckStream &cq, int nblk, int kk) {
    int *flag_copy = reinterpret_cast<int *>(chk + kChkFlag);
    BBL_HIP(hipMemcpyAsync(flag_copy, breakdown, sizeof(int), hipMemcpyDeviceToDevice, s));
    BBL_HIP(hipEventRecord(cq.ready, s));
    BBL_HIP(hipStreamWaitEvent(cq.cs, cq.ready, 0));
    const double *BJ = Bstore + (size_t)(nblk - 1) * b * b;
    if (time_eig_) BBL_HIP(hipEventRecord(cq.eig0, cq.cs));
    band_eigensolve(band, nblk * b, b, kk, eigws, L.el, BJ, b, S, chk, cq.cs);
    if (time_eig_) BBL_HIP(hipEventRecord(cq.eig1, cq.cs));
    eig_pending_ = time_eig_;
    BBL_HIP(hipMemcpyAsync(cq.host, chk, (2 * kk + 1) * sizeof(double), hipMemcpyDeviceToHost,
                           cq.cs));
    BBL_HIP(hipMemcpyAsync(cq.host + 2 * kMaxBlock + 4, flag_copy, sizeof(int),
                           hipMemcpyDeviceToHost, cq.cs));
    BBL_HIP(hipEventRecord(cq.done, cq.cs));
  }

  // Device time of the last launched check's band eigensolve (once it is done).
  bool time_eig_ = false, eig_pending_ = false;
  void harvest_eig(CheckStream &cq, Result &R) {
    if (!eig_pending_) return;
    eig_pending_ = false;
    float t = 0.f;
    BBL_HIP(hipEventSynchronize(cq.eig1));
    BBL_HIP(hipEventElapsedTime(&t, cq.eig0, cq.eig1));
    R.eig_ms += t;
  }

  // Reads the results of the check of nblk blocks (waiting for it if needed),
  // schedules the next one and, when the estimates pass (or `final`), forms
  // the Ritz vectors and their explicit residuals.  True when converged.
  bool consume_check(CheckStream &cq, int nblk, int kk, bool final, double *hnorm_dev,
                     double *Xout, Result &R) {
    fire_armed(cq);  // (a check is always launched before it is read)
    BBL_HIP(hipEventSynchronize(cq.done));
    harvest_eig(cq, R);
    const double *hres = cq.host;
    int flag = 0;
    std::memcpy(&flag, cq.host + 2 * kMaxBlock + 4, sizeof(int));
    if (flag) throw Error{BBL_E_BREAKDOWN, "block QR lost rank beyond deflation repair"};
    // ||H||_est for the block QRs queued from now on
    BBL_HIP(hipMemcpyAsync(hnorm_dev, chk + 2 * kk, sizeof(double), hipMemcpyDeviceToDevice, s));
    R.hnorm = hres[2 * kk];
    bool est_ok = true;
    double rho_max = 0.0;
    for (int i = 0; i < kk; ++i) {
      est_ok &= (hres[kk + i] <= tol * R.hnorm);
      rho_max = std::max(rho_max, hres[kk + i]);
    }
    next_check = next_check_after(nblk, rho_max, tol * R.hnorm);
    const bool exhausted = (int64_t)nblk * b >= n;
    if (!(exhausted || (kk == k && est_ok) || final)) return false;
    BBL_HIP(hipStreamWaitEvent(s, cq.done, 0));  // S of this check
    std::vector<double> r = ritz_and_residual(nblk, kk, Xout);
    ++R.spmm_calls;
    bool ok = kk == k || exhausted;
    for (int i = 0; i < kk; ++i) ok &= (r[i] <= tol * R.hnorm);
    R.theta.assign(hres, hres + kk);
    R.resid = r;
    R.iters = nblk;  // the returned pairs come from the first nblk blocks
    if (ok || exhausted) {
      R.converged = true;
      return true;
    }
    return false;
  }
  int next_check = 1;

  // Block QR of the fast path: the Cholesky factorisation only (its failure,
  // which the full path repairs with the spectral factor and deflation, is
  // recorded in chol_fail and makes the host redo the block).
  void block_qr_fast(int dest, double *Bout, const double *hnorm_dev, const double *Ov) {
    launch_chol_try(Ov, b, o.tau, hnorm_dev, dres + kHn2Slot, C0, QB, RB, mask, flag, chol_fail,
                    s);
    update_gram(Wp, BBL_F64, 1, 0, C0, 1.0, nullptr, BBL_F64, 0.0, Wp, O2, nullptr);
    launch_chol_finish(O2, b, RB, Rinv, Bout, breakdown, s);
    launch_update(n, Wp, BBL_F64, b, 1, 0, Rinv, b, 1.0, nullptr, BBL_F64, 0.0, slot(dest), xd,
                  s);
    ++qr_calls;
  }

  // Block J of the recurrence.  fast: the common path only -- one
  // Gram-Schmidt sweep and a Cholesky QR; whether the block needed a second
  // sweep (flag2) or a deflation repair (chol_fail) is copied to pinned
  // memory and read by the host one block later, and such a block is then
  // redone on the full path, which decides those branches on the device.
  void iterate(int J, bool fast, const double *hnorm_dev, PhaseTimer &timer, CheckStream &cq,
               Result &R) {
    if (fast)  // state as of this block's start, restored if it is redone:
      // max |A_jj|, and the sticky breakdown flag (an earlier block may have
      // raised it; the redone block's own QR decides again)
      launch_copy_pair(dres + kHn2Snap + J % kRing, dres + kHn2Slot, ints + kBreakSnap + J % kRing,
                       breakdown, s);
    hipEvent_t *ev = timer.begin();
    timer.mark(ev, 0, s);
    if (o.plan) launch_spmm_planned(*o.plan, slot(J), W, s);
    else launch_spmm(H, slot(J), xd, W, xd, b, s);
    timer.mark(ev, 1, s);
    ++R.spmm_calls;
    fire_armed(cq);
    gram(slot(J), xd, b, 1, 0, W, xd, b, Araw);
    launch_set_A(Araw, b, J, band, b, J > 0 ? Bstore + (size_t)(J - 1) * b * b : nullptr, C3,
                 dres + kHn2Slot, s);
    const int nb3 = J > 0 ? 2 : 1;
    update_gram(slot(J > 0 ? J - 1 : 0), xd, nb3, slot_stride(), C3, -1.0, W, xd, 1.0, Wp, G0,
                nullptr);
    timer.mark(ev, 2, s);
    double *BJ = Bstore + (size_t)J * b * b;
    if (fast) {
      gram(basis, xd, b, J + 1, slot_stride(), Wp, BBL_F64, b, C);
      update_gram(basis, xd, J + 1, slot_stride(), C, -1.0, Wp, BBL_F64, 1.0, Wp, G1, nullptr);
      launch_reorth_check(G0, G1, b, 0.5, nullptr, flag2, nullptr, s);
      // fault injection (testing): the block after the marked one needs a redo
      if (o.fault_block > 0 && J == o.fault_block) launch_store_int(flag2, 1, s);
      timer.mark(ev, 3, s);
      block_qr_fast(J + 1, BJ, hnorm_dev, G1);
      // fault injection (testing): the marked block's QR lost rank
      if (o.fault_block > 0 && J == o.fault_block - 1) launch_store_int(breakdown, 1, s);
    } else {
      reorth_recurrence(J + 1, Wp);
      timer.mark(ev, 3, s);
      block_qr(J + 1, J + 1, BJ, hnorm_dev, G1);
    }
    timer.mark(ev, 4, s);
    launch_set_B(BJ, b, J, band, b, o.m_max * b, s);
    if (fast) {  // flag2, n_second, chol_fail -> pinned slot J % kRing
      BBL_HIP(hipMemcpyAsync(cq.iter_flags(J), flag2, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
      BBL_HIP(hipEventRecord(cq.fev[J % kRing], s));
    }
  }

  // Thick restart after a cycle of nblk blocks (the next Lanczos block is in
  // slot nblk, B_{nblk-1} in the B store): the lowest p = restart_keep Ritz
  // pairs of the band matrix, the reduction of the arrowhead matrix they
  // form with the next block back to a band matrix (rotating the Ritz
  // vectors only), the rotated Ritz vectors Y' = V S_p Q formed in the spare
  // slots past m_max and moved to slots 0..p/b-1, and the next block moved to
  // slot p/b.  The recurrence then continues at block p/b unchanged: its
  // three-term step couples to the last block of Y' through B_{p/b-1}.
  void restart(int nblk, CheckStream &cq, Result &R) {
    const int p = o.restart_keep, q = p / b, N = nblk * b;
    double *rres = chk + 128;
    const double *Blast = Bstore + (size_t)(nblk - 1) * b * b;
    if (time_eig_) BBL_HIP(hipEventRecord(cq.rs0, s));
    band_eigensolve(band, N, b, p, eigws, L.el, Blast, b, S, rres, s);
    launch_restart_reduce(rres, S, p, (nblk - 1) * b, Blast, p, b, band, Bstore, Qr, s);
    launch_restart_coeffs(S, p, N, Qr, p, b, Sp, s);
    for (int j = 0; j < q; ++j)
      launch_update(n, basis, xd, b, nblk, slot_stride(), Sp + (size_t)j * N * b, b, 1.0, nullptr,
                    BBL_F64, 0.0, slot(o.m_max + 1 + j), xd, s);
    BBL_HIP(hipMemcpyAsync(slot(q), slot(nblk), (size_t)n * b * sx, hipMemcpyDeviceToDevice, s));
    BBL_HIP(hipMemcpyAsync(slot(0), slot(o.m_max + 1), (size_t)q * n * b * sx,
                           hipMemcpyDeviceToDevice, s));
    if (time_eig_) {
      BBL_HIP(hipEventRecord(cq.rs1, s));
      BBL_HIP(hipEventSynchronize(cq.rs1));
      float t = 0.f;
      BBL_HIP(hipEventElapsedTime(&t, cq.rs0, cq.rs1));
      R.restart_ms += t;
    }
    R.done_blocks += nblk - R.cycle_q;
    R.cycle_q = q;
    ++R.restarts;
    next_check = q + 1;
    have_prev_ = false;
  }

  Result run(const double *pivot, double *eigvecs_out) {
    Result R;
    CheckStreamLease lease(s);
    CheckStream &cq = *lease;
    // zero the band matrix, the B store, counters and results
    launch_fill(band, (int64_t)(o.m_max * b + b) * (b + 1), 0.0, s);
    launch_fill(Bstore, (int64_t)(o.m_max + 1) * b * b, 0.0, s);
    launch_fill(dres, 256, 0.0, s);
    launch_fill(reinterpret_cast<double *>(ints), 128, 0.0, s);
    double *hnorm_dev = dres + 2 * k;
    // V_1 from the pivot
    BBL_HIP(hipMemcpyAsync(Wp, pivot, (size_t)n * b * 8, hipMemcpyDeviceToDevice, s));
    block_qr(0, 0, Bstore + (size_t)o.m_max * b * b, hnorm_dev);
    double *Xout = eigvecs_out ? eigvecs_out : X;
    next_check = 1;
    int pending = 0, pending_kk = 0;  // blocks and pairs of the check in flight
    std::deque<int> unverified;       // fast blocks whose flags are not read yet
    int qr_snap[kRing] = {};          // qr_calls at the start of block J (J % kRing)
    const int check_lag = n < kShortRows ? kCheckLagShort : kLag;
    bool redo = false;
    PhaseTimer timer;
    timer.cq = &cq;
    timer.all_on = (o.flags & BBL_FLAG_TIME_PHASES) != 0;
    timer.spmm_on = timer.all_on || (o.flags & BBL_FLAG_TIME_SPMM) != 0;
    time_eig_ = timer.all_on;
    eig_pending_ = false;
    // Reads the flags of the unverified fast blocks up to `upto`, oldest
    // first (waiting for them).  At the first that needed a rare branch,
    // discards what followed it and returns it: that block is redone on the
    // full path.  Otherwise returns -1.
    auto verify = [&](int upto) {
      while (!unverified.empty() && unverified.front() <= upto) {
        const int U = unverified.front();
        unverified.pop_front();
        BBL_HIP(hipEventSynchronize(cq.fev[U % kRing]));
        const int *f = cq.iter_flags(U);
        if (!f[0] && !f[2]) continue;
        unverified.clear();
        if (pending) {  // its band matrix may contain discarded blocks
          armed_nblk_ = 0;
          BBL_HIP(hipStreamSynchronize(cq.cs));
          harvest_eig(cq, R);
          pending = 0;
        }
        BBL_HIP(hipMemcpyAsync(dres + kHn2Slot, dres + kHn2Snap + U % kRing, sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        // the breakdown flag is sticky: back to its value at the start of
        // block U (the discarded blocks did not count, earlier ones still do)
        BBL_HIP(hipMemcpyAsync(breakdown, ints + kBreakSnap + U % kRing, sizeof(int),
                               hipMemcpyDeviceToDevice, s));
        qr_calls = qr_snap[U % kRing];
        return U;
      }
      return -1;
    };
    int J = 0;
    while (J < o.m_max) {
      const bool fast = !redo;
      redo = false;
      qr_snap[J % kRing] = qr_calls;
      iterate(J, fast, hnorm_dev, timer, cq, R);
      R.iters = J + 1;
      R.built = std::max(R.built, J + 1);
      if (fast) unverified.push_back(J);
      // blocks kLag behind are read now: the queue still holds kLag blocks
      const int U = verify(J - kLag);
      if (U >= 0) {
        J = U;
        redo = true;
        continue;
      }
      // the pending check, once the block it ends with is verified
      const int ok_upto = unverified.empty() ? J : unverified.front() - 1;
      if (pending && pending - 1 <= ok_upto && J >= pending - 1 + check_lag) {
        const int nb = pending;
        pending = 0;
        if (consume_check(cq, nb, pending_kk, false, hnorm_dev, Xout, R)) break;
      }
      const int N = (J + 1) * b;
      const bool exhausted = (int64_t)N >= n;
      const bool last = (J == o.m_max - 1);
      const int kk = std::min(k, N);
      if (exhausted || last) {  // nothing left to overlap with: verify all, read now
        const int V = verify(J);
        if (V >= 0) {
          J = V;
          redo = true;
          continue;
        }
        if (pending) {
          const int nb = pending;
          pending = 0;
          if (consume_check(cq, nb, pending_kk, false, hnorm_dev, Xout, R)) break;
        }
        launch_check(cq, J + 1, kk);
        ++R.checks;
        const bool can_restart =
            o.restart_keep > 0 && !exhausted && R.restarts < o.max_restarts;
        if (consume_check(cq, J + 1, kk, !can_restart, hnorm_dev, Xout, R) || !can_restart)
          break;
        restart(J + 1, cq, R);
        J = o.restart_keep / b;
        continue;
      }
      // one check in flight at a time; a due check waits for the slot
      if (N >= k && J + 1 >= next_check && !pending) {
        arm_check(J + 1, kk);
        ++R.checks;
        pending = J + 1;
        pending_kk = kk;
      }
      ++J;
    }
    timer.finish();
    R.done_blocks += R.iters - R.cycle_q;  // all block iterations of all cycles
    R.spmm_ms = timer.ms[0];
    R.threeterm_ms = timer.ms[1];
    R.reorth_ms = timer.ms[2];
    R.qr_ms = timer.ms[3];
    R.spmm_timed = timer.spmm_on ? timer.spmm_count : 0;
    return R;
  }
};





// Kept Ritz vectors of a restarted truncated solve: the caller's restart_keep
// raised to cover the k wanted pairs (a multiple of b); the truncated-solve
// workspace always has room for the largest such value.
int trunc_keep(int keep, int b, int k) {
  if (keep <= 0) return 0;
  return std::max(keep, (int)ceil_div(std::max(k, b), b) * b);
}
int trunc_keep_max(int b, int k) {
  const int m = kMaxBlock / b * b;
  return m >= std::max(k, b) ? m : 0;
}

struct TruncLayout {
  size_t rp, col, val, piv, inner, total;
};

TruncLayout trunc_layout(int64_t n_t, int64_t nnz_t, int b, int k, int m_max, int bdt, int vdt) {
  TruncLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.rp = take((size_t)(n_t + 1) * 8);
  L.col = take((size_t)std::max<int64_t>(nnz_t, 1) * 4);
  L.val = take((size_t)std::max<int64_t>(nnz_t, 1) * dsize(vdt));
  L.piv = take((size_t)n_t * b * 8);
  L.inner = take(make_layout(n_t, b, k, m_max, bdt, trunc_keep_max(b, k)).total + 256);
  L.total = off + 256;
  return L;
}

}  // namespace

Opts read_opts(const bbl_opts *o, int val_dtype) {
  Opts r;
  if (o) {
    if (o->m_max > 0) r.m_max = o->m_max;
    r.basis_dtype = o->basis_dtype;
    r.check_every = o->check_every;
    r.flags = o->flags;
    r.plan = o->spmm_plan;
    r.restart_keep = o->restart_keep;
    r.max_restarts = o->max_restarts > 0 ? o->max_restarts : r.max_restarts;
    r.fault_block = o->fault_block;
    r.feature_vectors = o->feature_vectors;
    if (o->defl_tau > 0) r.tau = o->defl_tau;
    r.seed = o->seed;
  }
  if (r.basis_dtype == 0) r.basis_dtype = val_dtype;
  return r;
}


void validate_csr(const bbl_csr *H) {
  BBL_REQUIRE(H != nullptr, "H is NULL");
  BBL_REQUIRE(H->n >= 1, "H.n must be >= 1");
  BBL_REQUIRE(H->n <= (int64_t)INT32_MAX, "H.n exceeds int32 column range");
  BBL_REQUIRE(H->nnz >= 0, "H.nnz must be >= 0");
  BBL_REQUIRE(H->row_ptr && (H->nnz == 0 || (H->col && H->val)), "H has NULL arrays");
  BBL_REQUIRE(H->val_dtype == BBL_F32 || H->val_dtype == BBL_F64, "H.val_dtype must be F32/F64");
  BBL_REQUIRE(H->block_rows >= 0, "H.block_rows must be >= 0");
}


int64_t read_row_ptr(const bbl_csr &H, int64_t i, hipStream_t s) {
  int64_t v = 0;
  BBL_HIP(hipMemcpyAsync(&v, H.row_ptr + i, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BBL_HIP(hipStreamSynchronize(s));
  return v;
}


namespace {
void check_solver_args(const bbl_csr *H, int nvec, int k, const Opts &o) {
  validate_csr(H);
  BBL_REQUIRE(nvec >= 1 && nvec <= kMaxBlock, "nvec must be in 1..32");
  BBL_REQUIRE(k >= 1 && k <= kMaxBlock && (int64_t)k <= H->n, "k_eig must be in 1..min(n, 32)");
  BBL_REQUIRE(o.m_max >= 1, "m_max must be >= 1");
  BBL_REQUIRE((int64_t)k <= (int64_t)nvec * o.m_max, "k_eig exceeds nvec * m_max");
  BBL_REQUIRE(o.basis_dtype == BBL_F32 || o.basis_dtype == BBL_F64, "basis_dtype must be F32/F64");
  BBL_REQUIRE(!(o.basis_dtype == BBL_F32 && H->val_dtype == BBL_F64),
              "a float32 basis needs float32 matrix values");
  BBL_REQUIRE((int64_t)o.m_max * nvec <= 8192, "m_max * nvec must be <= 8192");
  BBL_REQUIRE(o.fault_block >= 0, "fault_block must be >= 0");
  BBL_REQUIRE(o.max_restarts >= 0, "max_restarts must be >= 0");
  if (o.restart_keep != 0)
    BBL_REQUIRE(o.restart_keep % nvec == 0 && o.restart_keep >= std::max(k, nvec) &&
                    o.restart_keep <= kMaxBlock && o.restart_keep / nvec + 1 < o.m_max,
                "restart_keep must be a multiple of nvec in [max(k_eig, nvec), "
                "min(32, nvec * (m_max - 2))]");
  if (o.plan) {
    BBL_REQUIRE(o.plan->n == H->n && o.plan->nnz == H->nnz && o.plan->row_ptr == H->row_ptr,
                "spmm_plan was built for another matrix");
    BBL_REQUIRE(o.plan->nvec == nvec && o.plan->vec_dtype == o.basis_dtype &&
                    o.plan->val_dtype == H->val_dtype,
                "spmm_plan nvec / vec_dtype must equal the block width and basis type");
  }
}
}  // namespace

int solve_impl(const bbl_csr *H, const double *pivot, int32_t nvec, int32_t k, double tol,
               void *ws, size_t ws_bytes, const Opts &o, double *eigvals, double *eigvecs,
               double *residuals, bbl_stats *stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  check_solver_args(H, nvec, k, o);
  BBL_REQUIRE(pivot != nullptr, "pivot is NULL");
  BBL_REQUIRE(ws != nullptr, "workspace is NULL");
  BBL_REQUIRE(eigvals != nullptr, "eigvals is NULL");
  BBL_REQUIRE(tol > 0.0, "tol must be > 0");
  Solver sv(*H, nvec, k, tol, o, ws, ws_bytes, s);
  Solver::Result R = sv.run(pivot, eigvecs);
  for (int i = 0; i < k; ++i) {
    eigvals[i] = i < (int)R.theta.size() ? R.theta[i] : NAN;
    if (residuals) residuals[i] = i < (int)R.resid.size() ? R.resid[i] : NAN;
  }
  int cnt[3] = {0, 0, 0};  // ndefl, flag2, n_second
  BBL_HIP(hipMemcpyAsync(cnt, sv.ndefl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  BBL_HIP(hipStreamSynchronize(s));
  const int nd = cnt[0];
  if (stats) {
    stats->iters = R.done_blocks;
    stats->basis_blocks = R.iters;
    stats->spmm_calls = R.spmm_calls;
    stats->deflations = nd;
    stats->converged = R.converged ? 1 : 0;
    stats->checks = R.checks;
    stats->reorth_second_passes = cnt[2];
    stats->hnorm_est = R.hnorm;
    stats->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stats->spmm_ms = R.spmm_ms;
    stats->spmm_timed = R.spmm_timed;
    stats->restarts = R.restarts;
    stats->t_threeterm_ms = R.threeterm_ms;
    stats->t_reorth_ms = R.reorth_ms;
    stats->t_qr_ms = R.qr_ms;
    stats->t_eig_ms = R.eig_ms;
    stats->t_restart_ms = R.restart_ms;
    stats->t_pivot_ms = 0.0;
    stats->pivot_spmm_calls = 0;
    stats->used_fallback = 0;
  }
  return R.converged ? BBL_OK : BBL_E_NOT_CONVERGED;
}

size_t truncated_ws_bytes(const bbl_csr &H, int64_t n_t, int b, int k, const Opts &o,
                          hipStream_t s) {
  const int bdt = o.basis_dtype ? o.basis_dtype : H.val_dtype;
  const int64_t nnz_t = read_row_ptr(H, n_t, s);
  return trunc_layout(n_t, nnz_t, b, k, o.m_max, bdt, H.val_dtype).total;
}

int truncated_solve(const bbl_csr &H, int64_t n_t, int b, int k, double tol, const Opts &o,
                    void *ws, size_t ws_bytes, double *eigvecs_t, double *theta,
                    bbl_stats *stats, hipStream_t s) {
  BBL_REQUIRE(n_t >= b && n_t >= k && n_t <= H.n, "truncation must be in max(nvec, k)..n");
  const int bdt = o.basis_dtype ? o.basis_dtype : H.val_dtype;
  const int64_t nnz_t = read_row_ptr(H, n_t, s);
  const TruncLayout L = trunc_layout(n_t, nnz_t, b, k, o.m_max, bdt, H.val_dtype);
  if (ws_bytes < L.total) throw Error{BBL_E_NOMEM, "truncated-solve workspace too small"};
  char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
  int64_t *rp_t = reinterpret_cast<int64_t *>(base + L.rp);
  int32_t *col_t = reinterpret_cast<int32_t *>(base + L.col);
  void *val_t = base + L.val;
  double *piv_t = reinterpret_cast<double *>(base + L.piv);
  launch_slice_leading(H, n_t, rp_t, col_t, val_t, s);
  bbl_csr Ht{};
  Ht.n = n_t;
  Ht.nnz = read_row_ptr(bbl_csr{n_t, 0, rp_t, nullptr, nullptr, BBL_F64, 0}, n_t, s);
  Ht.row_ptr = rp_t;
  Ht.col = col_t;
  Ht.val = val_t;
  Ht.val_dtype = H.val_dtype;
  Ht.block_rows = H.block_rows;
  // random pivot of the truncated problem, key (seed + 1) ^ golden ratio
  const uint64_t key = (o.seed + 1) ^ 0x9E3779B97F4A7C15ull;
  launch_gauss(n_t, b, b, 0, key, 6, piv_t, nullptr, nullptr, s);
  Opts oi = o;
  oi.seed = o.seed + 1;
  oi.basis_dtype = bdt;
  oi.plan = nullptr;  // the plan describes H, not its leading block
  oi.restart_keep = trunc_keep(o.restart_keep, b, k);
  return solve_impl(&Ht, piv_t, b, k, tol, base + L.inner, L.total - L.inner, oi, theta,
                    eigvecs_t, nullptr, stats, s);
}

namespace {

void check_band_eig_args(int N, int kd, int k) {
  BBL_REQUIRE(N >= 1 && N <= 8192 && kd >= 1 && kd <= kMaxBlock && k >= 1 &&
                  k <= std::min(N, kMaxBlock),
              "bad N/kd/k");
}

// The band eigensolve on a 256-byte aligned scratch region `base` of at least
// bbl_band_eig_workspace_size(N, kd, k) bytes: results at its start, the
// solver's workspace after them.
void band_eig_on(const double *band, int N, int kd, int k, char *base, double *theta, double *S,
                 double *top, hipStream_t s) {
  double *res = reinterpret_cast<double *>(base);
  const BandEigLayout L = band_eig_layout(N, kd, k);
  band_eigensolve(band, N, kd, k, base + 2 * 256 * 8, L, nullptr, kd, S, res, s);
  double h[2 * kMaxBlock + 2];
  BBL_HIP(hipMemcpyAsync(h, res, (2 * k + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
  BBL_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < k; ++i) theta[i] = h[i];
  if (top) *top = h[2 * k + 1];
}

// Scratch of bbl_band_eig_noalloc: a file-scope device array, so the call
// needs no allocation.  Every GPU the library runs on holds its own copy
// until the process ends; its device address is looked up once per device.
constexpr size_t kBandScratchBytes = (size_t)24 << 20;
__device__ __align__(256) unsigned char g_band_scratch[kBandScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

char *band_scratch_ptr() {
  int dev = 0;
  BBL_HIP(hipGetDevice(&dev));
  BBL_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    BBL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_band_scratch)));
    BBL_REQUIRE(p != nullptr, "no device address for the band-eigensolve scratch");
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

}  // namespace bbl

using namespace bbl;

extern "C" {

const char *bbl_last_error(void) { return g_last_error.c_str(); }

const char *bbl_version(void) { return "bbl 0.1 (gfx950)"; }

int bbl_spmm(const bbl_csr *H, const void *V, void *W, int32_t nvec, int32_t vec_dtype,
             void *stream) {
  return guarded([&] {
    validate_csr(H);
    BBL_REQUIRE(V && W, "V/W is NULL");
    BBL_REQUIRE(V != W, "V and W must not overlap");
    BBL_REQUIRE(nvec >= 1 && nvec <= kMaxBlock, "nvec must be in 1..32");
    BBL_REQUIRE(vec_dtype == BBL_F32 || vec_dtype == BBL_F64, "vec_dtype must be F32/F64");
    BBL_REQUIRE(!(vec_dtype == BBL_F32 && H->val_dtype == BBL_F64),
                "float32 vectors need float32 matrix values");
    launch_spmm(*H, V, vec_dtype, W, vec_dtype, nvec, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

size_t bbl_spmm_plan_size(const bbl_csr *H, int32_t nvec, int32_t vec_dtype) {
  size_t r = 0;
  const int st = guarded([&] {
    validate_csr(H);
    BBL_REQUIRE(vec_dtype == BBL_F32 || vec_dtype == BBL_F64, "vec_dtype must be F32/F64");
    r = spmm_plan_bytes(*H, nvec, vec_dtype);
    return (int)BBL_OK;
  });
  return st == BBL_OK ? r : 0;
}

int bbl_spmm_plan_build(const bbl_csr *H, int32_t nvec, int32_t vec_dtype, void *mem,
                        size_t bytes, bbl_spmm_plan *plan, void *stream) {
  return guarded([&] {
    validate_csr(H);
    BBL_REQUIRE(mem && plan, "mem/plan is NULL");
    BBL_REQUIRE(vec_dtype == BBL_F32 || vec_dtype == BBL_F64, "vec_dtype must be F32/F64");
    BBL_REQUIRE(vec_dtype == H->val_dtype, "plan: vector and value types must match");
    build_spmm_plan(*H, nvec, vec_dtype, mem, bytes, plan, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

int bbl_spmm_planned(const bbl_spmm_plan *plan, const void *V, void *W, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(plan && V && W, "NULL argument");
    BBL_REQUIRE(V != W, "V and W must not overlap");
    BBL_REQUIRE(plan->block_rows > 0 && plan->slots >= 1 && plan->slots <= kPlanMaxSlots &&
                    plan->blocks && plan->row_ptr &&
                    (plan->nsets > 0 ? (plan->sgroup && plan->srow && plan->slcol && plan->sval &&
                                        plan->rlist && plan->rgroup)
                                     : (plan->n_local && plan->col)),
                "plan is not initialised");
    launch_spmm_planned(*plan, V, W, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

size_t bbl_lanczos_workspace_size(int64_t n, int32_t nvec, int32_t k_eig, int32_t m_max,
                                  int32_t basis_dtype) {
  if (n < 1 || nvec < 1 || nvec > kMaxBlock || k_eig < 1 || k_eig > kMaxBlock || m_max < 1 ||
      (basis_dtype != BBL_F32 && basis_dtype != BBL_F64))
    return 0;
  return make_layout(n, nvec, k_eig, m_max, basis_dtype, 0).total;
}

size_t bbl_lanczos_workspace_size_restart(int64_t n, int32_t nvec, int32_t k_eig, int32_t m_max,
                                          int32_t basis_dtype, int32_t restart_keep) {
  if (bbl_lanczos_workspace_size(n, nvec, k_eig, m_max, basis_dtype) == 0 || restart_keep < 0 ||
      restart_keep > kMaxBlock || restart_keep % nvec)
    return 0;
  return make_layout(n, nvec, k_eig, m_max, basis_dtype, restart_keep).total;
}

int bbl_lanczos_workspace_views(const void *ws, int64_t n, int32_t nvec, int32_t k_eig,
                                int32_t m_max, int32_t basis_dtype, int32_t restart_keep,
                                void **basis, double **band) {
  return guarded([&] {
    BBL_REQUIRE(ws && basis && band, "NULL argument");
    BBL_REQUIRE(bbl_lanczos_workspace_size_restart(n, nvec, k_eig, m_max, basis_dtype,
                                                   restart_keep) > 0,
                "invalid sizes");
    const Layout L = make_layout(n, nvec, k_eig, m_max, basis_dtype, restart_keep);
    char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    *basis = base + L.basis;
    *band = reinterpret_cast<double *>(base + L.band);
    return (int)BBL_OK;
  });
}

int bbl_block_lanczos(const bbl_csr *H, const double *pivot, int32_t nvec, int32_t k_eig,
                      double tol, void *ws, size_t ws_bytes, const bbl_opts *opts,
                      double *eigvals, double *eigvecs, double *residuals, bbl_stats *stats,
                      void *stream) {
  return guarded([&] {
    BBL_REQUIRE(H != nullptr, "H is NULL");
    const Opts o = read_opts(opts, H->val_dtype);
    return solve_impl(H, pivot, nvec, k_eig, tol, ws, ws_bytes, o, eigvals, eigvecs, residuals,
                      stats, static_cast<hipStream_t>(stream));
  });
}

size_t bbl_bootstrap_workspace_size(const bbl_csr *H, int64_t n_trunc, int32_t nvec,
                                    int32_t m_max, int32_t basis_dtype, void *stream) {
  size_t r = 0;
  const int st = guarded([&] {
    validate_csr(H);
    BBL_REQUIRE(nvec >= 1 && nvec <= kMaxBlock, "nvec must be in 1..32");
    BBL_REQUIRE(n_trunc >= nvec && n_trunc <= H->n, "n_trunc must be in nvec..n");
    BBL_REQUIRE(m_max >= 1, "m_max must be >= 1");
    Opts o;
    o.m_max = m_max;
    o.basis_dtype = basis_dtype;
    r = truncated_ws_bytes(*H, n_trunc, nvec, nvec, o, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
  return st == BBL_OK ? r : 0;
}

int bbl_bootstrap_pivot(const bbl_csr *H, int64_t n_trunc, int32_t nvec, double tol, void *ws,
                        size_t ws_bytes, const bbl_opts *opts, double *pivot, bbl_stats *stats,
                        void *stream) {
  return guarded([&] {
    validate_csr(H);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BBL_REQUIRE(nvec >= 1 && nvec <= kMaxBlock, "nvec must be in 1..32");
    BBL_REQUIRE(n_trunc >= nvec && n_trunc <= H->n, "n_trunc must be in nvec..n");
    BBL_REQUIRE(pivot && ws, "pivot/workspace is NULL");
    const auto t0 = std::chrono::steady_clock::now();
    const Opts o = read_opts(opts, H->val_dtype);
    std::vector<double> ev(nvec);
    // the lowest nvec eigenvectors land in the first n_trunc rows of the pivot
    const int st = truncated_solve(*H, n_trunc, nvec, nvec, tol, o, ws, ws_bytes, pivot,
                                   ev.data(), stats, s);
    // zero padding: the truncated basis is a subset of the full one
    launch_fill(pivot + (size_t)n_trunc * nvec, (H->n - n_trunc) * nvec, 0.0, s);
    BBL_HIP(hipStreamSynchronize(s));
    if (stats) {
      stats->pivot_spmm_calls = stats->spmm_calls;
      stats->t_pivot_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
  });
}

size_t bbl_pivot_overlap_workspace_size(int64_t n, int32_t k, int32_t nvec) {
  if (n < 1 || k < 1 || k > kMaxBlock || nvec < 1 || nvec > kMaxBlock) return 0;
  return gram_partial_doubles(std::max(k, nvec), nvec) * 8 + 8 * 1024 * 8 + 512;
}

int bbl_pivot_overlap(int64_t n, const double *X, int32_t k, const double *P, int32_t nvec,
                      void *ws, size_t ws_bytes, double *cosines, double *captured,
                      void *stream) {
  return guarded([&] {
    BBL_REQUIRE(X && P && ws && cosines, "NULL argument");
    const size_t need = bbl_pivot_overlap_workspace_size(n, k, nvec);
    BBL_REQUIRE(need > 0, "bad n/k/nvec");
    if (ws_bytes < need) throw Error{BBL_E_NOMEM, "overlap workspace too small"};
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    double *M = reinterpret_cast<double *>(base);
    double *G = M + 2 * 1024;
    double *out = G + 2 * 1024;
    double *partial = reinterpret_cast<double *>(base + 8 * 1024 * 8);
    const size_t pcap = (need - 512 - 8 * 1024 * 8) / 8;
    int P1 = launch_gram(n, X, BBL_F64, k, 1, 0, P, BBL_F64, nvec, partial,
                         gram_max_partials(pcap, k, nvec), s);
    launch_reduce(partial, P1, k, nvec, M, s);
    P1 = launch_gram(n, P, BBL_F64, nvec, 1, 0, P, BBL_F64, nvec, partial,
                     gram_max_partials(pcap, nvec, nvec), s);
    launch_reduce(partial, P1, nvec, nvec, G, s);
    launch_overlap(M, G, k, nvec, out, s);
    double h[2 * kMaxBlock];
    BBL_HIP(hipMemcpyAsync(h, out, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s));
    BBL_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < k; ++i) {
      cosines[i] = h[i];
      if (captured) captured[i] = h[k + i];
    }
    return (int)BBL_OK;
  });
}

int bbl_random_pivot(int64_t n, int32_t nvec, uint64_t key, double *pivot, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(n >= 1 && nvec >= 1 && nvec <= kMaxBlock, "bad n/nvec");
    BBL_REQUIRE(pivot != nullptr, "pivot is NULL");
    launch_gauss(n, nvec, nvec, 0, key, 6, pivot, nullptr, nullptr,
                 static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

size_t bbl_band_eig_workspace_size(int32_t N, int32_t kd, int32_t k) {
  if (N < 1 || kd < 1 || kd > kMaxBlock || k < 1 || k > kMaxBlock || k > N || N > 8192) return 0;
  return band_eig_layout(N, kd, k).bytes + 2 * 256 * 8 + 256;
}

int bbl_band_eig(const double *band, int32_t N, int32_t kd, int32_t k, void *ws, size_t ws_bytes,
                 double *theta, double *S, double *top, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(band && ws && theta && S, "NULL argument");
    check_band_eig_args(N, kd, k);
    const size_t need = bbl_band_eig_workspace_size(N, kd, k);
    if (ws_bytes < need) throw Error{BBL_E_NOMEM, "band eig workspace too small"};
    band_eig_on(band, N, kd, k, reinterpret_cast<char *>(align_up(reinterpret_cast<uintptr_t>(ws), 256)),
                theta, S, top, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

int bbl_band_eig_noalloc(const double *band, int32_t N, int32_t kd, int32_t k, double *theta,
                         double *S, double *top, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(band && theta && S, "NULL argument");
    check_band_eig_args(N, kd, k);
    const size_t need = bbl_band_eig_workspace_size(N, kd, k);
    if (need > kBandScratchBytes)
      throw Error{BBL_E_INVALID, "band eig without allocation: N, kd, k need " +
                                     std::to_string(need) + " bytes of scratch, more than the " +
                                     std::to_string(kBandScratchBytes) + " the library holds"};
    band_eig_on(band, N, kd, k, band_scratch_ptr(), theta, S, top,
                static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

size_t bbl_gram_workspace_size(int64_t n, int32_t bx, int32_t nblk, int32_t ny) {
  if (n < 1 || bx < 1 || nblk < 1 || ny < 1 || ny > kMaxBlock) return 0;
  return gram_partial_doubles((int64_t)bx * nblk, ny) * 8 + 512;
}

int bbl_gram(int64_t n, const void *X, int32_t xdtype, int32_t bx, int32_t nblk, const void *Y,
             int32_t ydtype, int32_t ny, double *C, void *ws, size_t ws_bytes, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(X && Y && C && ws, "NULL argument");
    BBL_REQUIRE(n >= 1 && bx >= 1 && nblk >= 1 && ny >= 1 && ny <= kMaxBlock, "bad sizes");
    BBL_REQUIRE((xdtype == BBL_F32 || xdtype == BBL_F64) && (ydtype == BBL_F32 || ydtype == BBL_F64),
                "bad dtype");
    const size_t need = bbl_gram_workspace_size(n, bx, nblk, ny);
    if (ws_bytes < need) throw Error{BBL_E_NOMEM, "gram workspace too small"};
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *partial = reinterpret_cast<double *>(align_up(reinterpret_cast<uintptr_t>(ws), 256));
    const int M = bx * nblk;
    const int maxp = gram_max_partials((need - 512) / 8, M, ny);
    const int P = launch_gram(n, X, xdtype, bx, nblk, n * bx, Y, ydtype, ny, partial, maxp, s);
    launch_reduce(partial, P, M, ny, C, s);
    return (int)BBL_OK;
  });
}

int bbl_block_update(int64_t n, const void *X, int32_t xdtype, int32_t bx, int32_t nblk,
                     const double *C, int32_t ny, double alpha, const void *Yin, int32_t yindtype,
                     double beta, void *Yout, int32_t youtdtype, void *stream) {
  return guarded([&] {
    BBL_REQUIRE(X && C && Yout && (beta == 0.0 || Yin), "NULL argument");
    BBL_REQUIRE(n >= 1 && bx >= 1 && nblk >= 1 && ny >= 1 && ny <= kMaxBlock, "bad sizes");
    BBL_REQUIRE(!(X == Yout && nblk != 1), "in-place X == Yout needs nblk == 1");
    launch_update(n, X, xdtype, bx, nblk, n * bx, C, ny, alpha, Yin, yindtype, beta, Yout,
                  youtdtype, static_cast<hipStream_t>(stream));
    return (int)BBL_OK;
  });
}

}  // extern "C"
