// Seeded synthetic input generator: sectored "shell-model-shaped" symmetric
// sparse matrices and Gaussian blocks.  Both the HIP path and the CPU oracle
// take their inputs from here; nothing in this file performs any step of the
// eigensolver itself (no products with H, no orthogonalisation, no solves).
//
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), written here from its
// published definition.  Every draw is addressed by a counter, so the output
// is identical for any thread count.
//
// Matrix recipe (a synthetic stand-in for the M-scheme Hamiltonians of the
// paper's Results section, whose basis is blocked by Abelian quantum numbers,
// Appendix A):
//   * n rows in S = n / R contiguous "sectors" of R rows;
//   * diagonal = the order statistics of n iid U(-40, 40) draws plus
//     N(0, 0.5^2) noise, so leading rows carry the lowest unperturbed
//     energies (the analogue of a W <= W_max truncation);
//   * each sector couples to 3 distinct partner sectors;
//   * each row draws q columns: with probability p uniform in its own sector,
//     otherwise uniform in one of its sector's 3 partners; value N(0, 1);
//     the draw j == i is dropped;
//   * every draw (i, j, v) is stored at (i, j) and (j, i); duplicates are summed
//     in ascending-value order, so the result is exactly symmetric and does not
//     depend on the order of the parallel fill.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>
#include <omp.h>

namespace {

struct U4 { uint32_t v[4]; };

inline void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

// Philox4x32 with 10 rounds: S-box = two 32x32->64 multiplies, key schedule
// bumped by the Weyl constants between rounds.
inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo(M0, c.v[0], hi0, lo0);
    mulhilo(M1, c.v[2], hi1, lo1);
    U4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
  }
  return c;
}

inline U4 draw(uint64_t key, uint64_t a, uint32_t b, uint32_t tag) {
  U4 c;
  c.v[0] = (uint32_t)a;
  c.v[1] = (uint32_t)(a >> 32);
  c.v[2] = b;
  c.v[3] = tag;
  return philox4x32_10(c, (uint32_t)key, (uint32_t)(key >> 32));
}

// 53-bit uniform in the open interval (0, 1) from two 32-bit words.
inline double u53(uint32_t hi, uint32_t lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

// Box-Muller (cosine branch) from one Philox output.
inline double gauss(const U4& w) {
  const double u1 = u53(w.v[0], w.v[1]);
  const double u2 = u53(w.v[2], w.v[3]);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925 * u2);
}

// Stream tags (the fourth counter word) keep the uses of one key apart.
enum : uint32_t {
  TAG_DIAG_SPACING = 1,
  TAG_DIAG_NOISE = 2,
  TAG_PARTNER = 3,
  TAG_DRAW_CHOICE = 4,
  TAG_DRAW_VALUE = 5,
  TAG_GAUSS_BLOCK = 6,
};

struct Params {
  int64_t n, R;
  int32_t q;
  double p;
  uint64_t seed;
  int verbose;  // progress lines on stderr after each pass
};

double now_s() { return omp_get_wtime(); }
void progress(const Params& P, const char* what, double t0) {
  if (P.verbose) {
    std::fprintf(stderr, "[synthgen] n=%lld: %s (%.1f s)\n", (long long)P.n, what, now_s() - t0);
    std::fflush(stderr);
  }
}

inline uint32_t umul_range(uint32_t w, uint64_t range) {  // floor(w * range / 2^32)
  return (uint32_t)(((uint64_t)w * range) >> 32);
}

// Column drawn by row i at draw t, or -1 when the draw is j == i; its value
// into *val unless val is NULL.
inline int64_t draw_col(const Params& P, const int32_t* partners, int64_t i, int32_t t, double* val) {
  const int64_t s = i / P.R;
  const U4 w = draw(P.seed, (uint64_t)i, (uint32_t)t, TAG_DRAW_CHOICE);
  const uint64_t thr = (uint64_t)std::llround(P.p * 4294967296.0);
  int64_t tgt;
  if ((uint64_t)w.v[0] < thr) {
    tgt = s;
  } else {
    tgt = partners[3 * s + umul_range(w.v[1], 3)];
  }
  const int64_t j = tgt * P.R + (int64_t)umul_range(w.v[2], (uint64_t)P.R);
  if (j == i) return -1;
  if (val) *val = gauss(draw(P.seed, (uint64_t)i, (uint32_t)t, TAG_DRAW_VALUE));
  return j;
}

// The assembled matrix: row i's ucnt[i] entries (sorted, duplicates summed)
// sit at tcol/tval[p0[i] ..] with gaps between rows; sg_export compacts them
// straight into the caller's arrays, so the largest instances never hold a
// second full copy.
struct Matrix {
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> row_ptr, p0;
  std::vector<int32_t> tcol;
  std::vector<double> tval;
  std::vector<double> diag;
  std::vector<int32_t> partners;
};

// Deterministic prefix sum over fixed-size chunks (independent of threads).
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n) {
  const int64_t CH = 1 << 16;
  const int64_t nch = (n + CH - 1) / CH;
  std::vector<int64_t> part(nch + 1, 0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    int64_t s = 0;
    const int64_t e = std::min(n, (c + 1) * CH);
    for (int64_t i = c * CH; i < e; ++i) s += in[i];
    part[c + 1] = s;
  }
  for (int64_t c = 0; c < nch; ++c) part[c + 1] += part[c];
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    int64_t s = part[c];
    const int64_t e = std::min(n, (c + 1) * CH);
    for (int64_t i = c * CH; i < e; ++i) { out[i] = s; s += in[i]; }
  }
  out[n] = part[nch];
}

void make_diag(const Params& P, std::vector<double>& d) {
  // Order statistics of n iid U(0,1): u_(i) = S_i / S_{n+1}, S_i the partial
  // sums of n+1 iid Exp(1) spacings.  Same joint law as sorting n uniforms.
  const int64_t n = P.n;
  std::vector<double> e(n + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i <= n; ++i) {
    const U4 w = draw(P.seed, (uint64_t)i, 0u, TAG_DIAG_SPACING);
    e[i] = -std::log(u53(w.v[0], w.v[1]));
  }
  // deterministic chunked prefix sum in double
  const int64_t CH = 1 << 16;
  const int64_t nch = (n + 1 + CH - 1) / CH;
  std::vector<double> part(nch + 1, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    double s = 0.0;
    const int64_t end = std::min(n + 1, (c + 1) * CH);
    for (int64_t i = c * CH; i < end; ++i) s += e[i];
    part[c + 1] = s;
  }
  for (int64_t c = 0; c < nch; ++c) part[c + 1] += part[c];
  const double total = part[nch];
  d.resize(n);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    double s = part[c];
    const int64_t end = std::min(n, (c + 1) * CH);
    for (int64_t i = c * CH; i < end; ++i) {
      s += e[i];
      const double u = s / total;
      const double z = gauss(draw(P.seed, (uint64_t)i, 0u, TAG_DIAG_NOISE));
      d[i] = -40.0 + 80.0 * u + 0.5 * z;
    }
  }
}

void make_partners(const Params& P, std::vector<int32_t>& partners) {
  const int64_t S = P.n / P.R;
  partners.assign(3 * S, 0);
  if (S < 2) return;  // a single sector couples only to itself
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S; ++s) {
    int32_t got[3];
    int ng = 0;
    for (uint32_t attempt = 0; ng < 3; ++attempt) {
      const U4 w = draw(P.seed, (uint64_t)s, attempt, TAG_PARTNER);
      for (int k = 0; k < 4 && ng < 3; ++k) {
        // uniform over the other S - 1 sectors
        int64_t c = umul_range(w.v[k], (uint64_t)(S - 1));
        if (c >= s) ++c;
        bool dup = false;
        for (int m = 0; m < ng; ++m) dup |= (got[m] == (int32_t)c);
        // fewer than 3 other sectors exist: allow repeats
        if (dup && S - 1 >= 3) continue;
        got[ng++] = (int32_t)c;
      }
    }
    for (int k = 0; k < 3; ++k) partners[3 * s + k] = got[k];
  }
}

Matrix* build(const Params& P) {
  const double t0 = now_s();
  Matrix* M = new Matrix();
  M->n = P.n;
  make_diag(P, M->diag);
  make_partners(P, M->partners);
  const int32_t* partners = M->partners.data();
  const int64_t n = P.n;

  // pass 1: counts
  std::vector<std::atomic<int64_t>> cnt(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) cnt[i].store(1, std::memory_order_relaxed);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t t = 0; t < P.q; ++t) {
      const int64_t j = draw_col(P, partners, i, t, nullptr);
      if (j < 0) continue;
      cnt[i].fetch_add(1, std::memory_order_relaxed);
      cnt[j].fetch_add(1, std::memory_order_relaxed);
    }
  }
  progress(P, "draws counted", t0);
  std::vector<int64_t> c0(n);
  std::vector<int64_t>& p0 = M->p0;
  p0.resize(n + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) c0[i] = cnt[i].load(std::memory_order_relaxed);
  exclusive_scan_i64(c0.data(), p0.data(), n);
  { std::vector<int64_t>().swap(c0); }
  const int64_t tot = p0[n];

  // pass 2: fill (order within a row is arbitrary here; fixed by the sort)
  std::vector<int32_t>& tcol = M->tcol;
  std::vector<double>& tval = M->tval;
  tcol.resize(tot);
  tval.resize(tot);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    tcol[p0[i]] = (int32_t)i;
    tval[p0[i]] = M->diag[i];
    cnt[i].store(p0[i] + 1, std::memory_order_relaxed);
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t t = 0; t < P.q; ++t) {
      double v;
      const int64_t j = draw_col(P, partners, i, t, &v);
      if (j < 0) continue;
      const int64_t a = cnt[i].fetch_add(1, std::memory_order_relaxed);
      tcol[a] = (int32_t)j;
      tval[a] = v;
      const int64_t b = cnt[j].fetch_add(1, std::memory_order_relaxed);
      tcol[b] = (int32_t)i;
      tval[b] = v;
    }
  }
  { std::vector<std::atomic<int64_t>>().swap(cnt); }
  progress(P, "draws placed", t0);

  // pass 3: per-row sort by (col, value), sum duplicates in that order
  std::vector<int64_t> ucnt(n);
#pragma omp parallel
  {
    std::vector<std::pair<int32_t, double>> buf;
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t b = p0[i], e = p0[i + 1];
      buf.resize(e - b);
      for (int64_t k = b; k < e; ++k) buf[k - b] = {tcol[k], tval[k]};
      std::sort(buf.begin(), buf.end());
      int64_t u = 0;
      for (size_t k = 0; k < buf.size(); ++k) {
        if (u > 0 && tcol[b + u - 1] == buf[k].first) {
          tval[b + u - 1] += buf[k].second;
        } else {
          tcol[b + u] = buf[k].first;
          tval[b + u] = buf[k].second;
          ++u;
        }
      }
      ucnt[i] = u;
    }
  }
  M->row_ptr.resize(n + 1);
  exclusive_scan_i64(ucnt.data(), M->row_ptr.data(), n);
  M->nnz = M->row_ptr[n];
  progress(P, "rows sorted and merged", t0);
  return M;
}

}  // namespace

extern "C" {

// Builds the matrix; returns an opaque handle (NULL on bad arguments or OOM).
void* sg_generate(int64_t n, int64_t R, int32_t q, double p, uint64_t seed, int32_t nthreads,
                  int32_t verbose) {
  if (n < 1 || R < 1 || n % R != 0 || q < 0 || p < 0.0 || p > 1.0) return nullptr;
  if (n > (int64_t)INT32_MAX) return nullptr;  // column indices are int32
  if (nthreads > 0) omp_set_num_threads(nthreads);
  Params P{n, R, q, p, seed, verbose};
  try {
    return build(P);
  } catch (const std::bad_alloc&) {
    return nullptr;
  }
}

int64_t sg_nnz(void* h) { return static_cast<Matrix*>(h)->nnz; }

// Copies the CSR arrays out (row_ptr[n+1], col[nnz], val[nnz]); any pointer may
// be NULL to skip it.  val32 receives the values rounded to float.
void sg_export(void* h, int64_t* row_ptr, int32_t* col, double* val, float* val32, double* diag,
               int32_t* partners) {
  Matrix* M = static_cast<Matrix*>(h);
  const int64_t n = M->n;
  if (row_ptr) std::memcpy(row_ptr, M->row_ptr.data(), sizeof(int64_t) * (n + 1));
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t src = M->p0[i], dst = M->row_ptr[i], len = M->row_ptr[i + 1] - dst;
    if (col) std::memcpy(col + dst, &M->tcol[src], sizeof(int32_t) * len);
    if (val) std::memcpy(val + dst, &M->tval[src], sizeof(double) * len);
    if (val32)
      for (int64_t k = 0; k < len; ++k) val32[dst + k] = (float)M->tval[src + k];
  }
  if (diag) std::memcpy(diag, M->diag.data(), sizeof(double) * M->n);
  if (partners) std::memcpy(partners, M->partners.data(), sizeof(int32_t) * M->partners.size());
}

void sg_free(void* h) { delete static_cast<Matrix*>(h); }

// Gaussian block G[n][b] (row-major), entry (i, a) from counter (i, a, tag 6).
void sg_gaussian_block(int64_t n, int32_t b, uint64_t key, double* out, int32_t nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int32_t a = 0; a < b; ++a)
      out[i * b + a] = gauss(draw(key, (uint64_t)i, (uint32_t)a, TAG_GAUSS_BLOCK));
}

// Raw Philox4x32-10 words for known-answer and cross-implementation checks.
void sg_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  U4 c;
  for (int k = 0; k < 4; ++k) c.v[k] = ctr[k];
  const U4 o = philox4x32_10(c, key[0], key[1]);
  for (int k = 0; k < 4; ++k) out[k] = o.v[k];
}

}  // extern "C"
