// Internal declarations of the PCV library: context, device buffers and the
// device-side building blocks shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pcv.h"

namespace pcv {

constexpr uint32_t TAG_MOMENTUM = 1;
constexpr uint32_t TAG_ACCEPT = 2;
constexpr uint32_t TAG_SHUFFLE = 3;
constexpr uint32_t TAG_PREDICT = 4;   // predictive draws of the test rows (DSS)
constexpr uint32_t TAG_INIT = 5;      // starting draw of a chain from the full-data draws
constexpr double DIVERGENCE_THRESHOLD = 1000.0;
constexpr int MAX_BLOCKS = 64;

// Post-hoc statistics of one fold's stored draws s[l * N + i] (host code,
// posthoc.hip): log fhat, pooled and batch-means variances of f = e^s relative
// to fhat^2, and the paper's, split and rank-normalised split R-hats.
struct PosthocFold {
  double log_fhat, s2rel, sig2rel, rhat, split_rhat, rank_rhat;
};
void posthoc_fold(const double* s, int L, int64_t N, int b, PosthocFold& out);

// ----------------------------------------------------------------------------
// Kernel argument bundle (plain device pointers; passed by value).
// ----------------------------------------------------------------------------
struct DevModel {
  int family, fold_kind;
  int64_t n, p, d, C;
  int K, L, n_groups;
  // models in one launch (Appendix B): M models x K folds = KP posteriors,
  // model-major; mmask [M][p] (1 = covariate used), null for one model
  int M, KP;
  const uint8_t* mmask;
  double sigma, inv_sigma2, eps;
  int S;
  int64_t n_warmup;
  int b, Gb, D;
  uint32_t key0, key1;
  int64_t chain_offset;
  // data
  const double* X64;      // [n][p]
  const float* X32;       // [n][p] (fp32 VALU path)
  const double* y64;      // [n]
  const float* y32;       // [n]
  const double* rowc;     // [n] per-row log-likelihood constant
  const int32_t* fold_index;  // INDEX [n]
  const int32_t* ivals;       // INTERVALS [K][4]
  const int8_t* roles;        // DENSE [K][n]
  const int32_t* test_ptr;    // [K+1]
  const int32_t* test_rows;   // [nnz]
  const int32_t* group_of;    // HIER [n]
  const int32_t* wave_rows;   // VALU row partition [W+1] ([splits][W+1] on the row-split path)
  const int32_t* gsplit;      // HIER row splits: first and last split spanning group g, [G][2]
  const double* minv;         // [d]
  const double* prior_prec;   // [d] 1/scale^2
  const double* fold_const;   // [K]
  const double* ntrain;       // [K] training rows per fold (FAM_HGAUSS: the -n log sigma_y term)
  // chain state, [d][C] (chain index fastest)
  double *q0, *g0, *q1, *g1, *pm;
  double *logp0, *logp1, *s0, *h0;
  // accumulators.  Block statistics: Welford mean and M2 of s, or with
  // rhat_mode 1 (shifted sums) sum (s - C_k) and sum (s - C_k)^2
  double *Z, *U, *U2, *V, *V2, *bmean, *bm2;   // [C], [D][C]
  int64_t *nacc, *ndiv;
  int rhat_mode;
  double* wsum;     // [C] sum of warm-up draws of s (shifted sums)
  double* center;   // [K] C_k, the fold's warm-up mean of s (shifted sums)
  // Hyvaerinen / Dawid-Sebastiani scores (bit mask: 1 HS, 2 DSS).  Per chain
  // c = k L + l, test-row slot a of its fold: [L * test_ptr[k] + l v_k + a];
  // per row pair (a, b): [L * sq_ptr[k] + l v_k^2 + a v_k + b].
  int scores;
  double* hs1;      // [C] sum over draws and test rows of d2 + d1^2
  double* hs2;      // [L nnz] sum over draws of d1 per test row
  double* dx;       // [L nnz] sum over draws of (ytil - y)
  double* dxx;      // [L sum_k v_k^2] sum over draws of (ytil_a - y_a)(ytil_b - y_b)
  double* rcur;     // [L nnz] this draw's ytil - y (scratch)
  const int64_t* sq_ptr;  // [K+1]
  // stored post-warm-up draws of s (Algorithm 1): draw i of chain c at [i C + c]
  double* draws;
  int64_t draws_cap;
  // device-side transition counter (read when a kernel is given t < 0, so
  // one captured graph of a transition can be replayed)
  int64_t* t_dev;
  // [C] acceptance statistic min(1, e^(H0 - H1)) of the last transition (0
  // for a non-finite energy); read by the window adaptation
  double* acc_stat;
  // split paths: log predictive of the proposal q1 over the fold's test rows,
  // in lp_groups partial sums per chain ([lp_groups][C], k_testlp), added by
  // k_accept; null when the folds' test rows are few enough for k_accept's
  // own loop
  double* lp_part;
  int lp_groups;
};

// ----------------------------------------------------------------------------
// Device helpers
// ----------------------------------------------------------------------------
struct W4 {
  uint32_t x, y, z, w;
};

// Philox4x32 with ten rounds (Salmon et al., SC'11); also used on the host.
__host__ __device__ __forceinline__ W4 philox4x32_10(W4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
    c = W4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Two 32-bit words -> double strictly inside (0,1): top 52 bits, centred in their cell.
__host__ __device__ __forceinline__ double uniform01(uint32_t w0, uint32_t w1) {
  const uint64_t b = (static_cast<uint64_t>(w0) << 32) | w1;
  return static_cast<double>(b >> 12) * 0x1p-52 + 0x1p-53;
}

__device__ __forceinline__ double log_add_exp(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  const double m = a > b ? a : b;
  return m + log1p(exp(-fabs(a - b)));
}

enum { FAM_GAUSS = 0, FAM_LOGIT = 1, FAM_POIS = 2, FAM_HIER = 3, FAM_HGAUSS = 4 };
// Hierarchical families: theta = [beta (p), mu, log group scale, (log sigma_y,) z (groups)],
// eta = x'beta + mu + e^{log group scale} z_g.  FAM_HIER: Bernoulli-logit;
// FAM_HGAUSS: Gaussian with unknown noise sd sigma_y = e^{theta[p + 2]}.
template <int FAM>
__host__ __device__ constexpr bool hier_fam() { return FAM == FAM_HIER || FAM == FAM_HGAUSS; }
__host__ __device__ constexpr bool hier_family(int fam) { return fam == FAM_HIER || fam == FAM_HGAUSS; }
// variance of the half-normal priors of the two scales of FAM_HGAUSS
constexpr double HGAUSS_SCALE_VAR = 10.0;
// MFMA tile shapes of the matrix-core gradient kernel (a launch-shape knob)
// (MFMA_SHAPE_32X32X16_IL: the 32x32x16 kernel scheduled by the compiler across groups)
// (MFMA_SHAPE_16X16X32_C16: the 16x16x32 kernel with 16 chains per wave, two
// workgroups per CU; design widths p <= 64 only)
enum { MFMA_SHAPE_16X16X32 = 0, MFMA_SHAPE_32X32X16 = 1, MFMA_SHAPE_32X32X16_IL = 2, MFMA_SHAPE_16X16X32_C16 = 3 };

// d l(y, eta) / d eta and l(y, eta) minus its per-row constant.
// (FAM_HGAUSS: the Gaussian forms with the chain's own 1/sigma_y^2; its
// per-row -log sigma_y is added by the callers.)
template <int FAM>
__device__ __forceinline__ double resid64(double y, double eta, double inv_sigma2) {
  if (FAM == FAM_GAUSS || FAM == FAM_HGAUSS) return (y - eta) * inv_sigma2;
  if (FAM == FAM_POIS) return y - exp(eta);
  return y - 1.0 / (1.0 + exp(-eta));
}
template <int FAM>
__device__ __forceinline__ double ell0_64(double y, double eta, double inv_sigma2) {
  if (FAM == FAM_GAUSS || FAM == FAM_HGAUSS) {
    const double e = y - eta;
    return -0.5 * e * e * inv_sigma2;
  }
  if (FAM == FAM_POIS) return y * eta - exp(eta);
  return y * eta - (fmax(eta, 0.0) + log1p(exp(-fabs(eta))));
}
template <int FAM>
__device__ __forceinline__ float resid32(float y, float eta, float inv_sigma2) {
  if (FAM == FAM_GAUSS || FAM == FAM_HGAUSS) return (y - eta) * inv_sigma2;
  if (FAM == FAM_POIS) return y - __expf(eta);
  return y - 1.0f / (1.0f + __expf(-eta));
}
template <int FAM>
__device__ __forceinline__ float ell0_32(float y, float eta, float inv_sigma2) {
  if (FAM == FAM_GAUSS || FAM == FAM_HGAUSS) {
    const float e = y - eta;
    return -0.5f * e * e * inv_sigma2;
  }
  if (FAM == FAM_POIS) return y * eta - __expf(eta);
  return y * eta - (fmaxf(eta, 0.0f) + log1pf(__expf(-fabsf(eta))));
}

// Data fold of chain c (its posterior index modulo the folds), and the row
// of the covariate mask of its model (null with one model: every covariate
// used).  Chain indices fit 32 bits (checked at init), so the divisions are
// 32-bit; call these once per chain, outside loops over rows or covariates.
// First z coordinate of the hierarchical families.
__host__ __device__ __forceinline__ int64_t hier_z0(const DevModel& m) {
  return m.p + (m.family == FAM_HGAUSS ? 3 : 2);
}
__host__ __device__ __forceinline__ int fold_of_chain(const DevModel& m, int64_t c) {
  const uint32_t post = static_cast<uint32_t>(c) / static_cast<uint32_t>(m.L);
  return static_cast<int>(m.M > 1 ? post % static_cast<uint32_t>(m.K) : post);
}
__device__ __forceinline__ const uint8_t* mask_row(const DevModel& m, int64_t c) {
  if (!m.mmask) return nullptr;
  const uint32_t model = static_cast<uint32_t>(c) / static_cast<uint32_t>(m.L * m.K);
  return m.mmask + static_cast<int64_t>(model) * m.p;
}
__device__ __forceinline__ bool covariate_used(const uint8_t* row, int64_t j) { return !row || row[j] != 0; }

// Coefficients j < PB of chain c at position q ([d][C]), zero at j >= p and
// where the chain's model drops j.  Every load is unconditional (clamped
// index; the selection comes after), so all of them are in flight at once: a
// load under a per-lane condition compiles to a branch that waits for that
// load alone.
template <int PB, typename T>
__device__ __forceinline__ void theta_row(const DevModel& m, const double* q, int64_t c, T (&th)[PB]) {
  double tv[PB];
  bool keep[PB];
#pragma unroll
  for (int j = 0; j < PB; ++j) {
    tv[j] = q[(j < m.p ? j : m.p - 1) * m.C + c];
    keep[j] = j < m.p;
  }
  if (m.mmask) {
    const uint8_t* mrow = mask_row(m, c);
    uint8_t mb[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) mb[j] = mrow[j < m.p ? j : m.p - 1];
#pragma unroll
    for (int j = 0; j < PB; ++j) keep[j] = keep[j] && mb[j] != 0;
  }
#pragma unroll
  for (int j = 0; j < PB; ++j) th[j] = keep[j] ? static_cast<T>(tv[j]) : T(0);
}

// Role of row i in fold k: 0 excluded, 1 train, 2 test.
__device__ __forceinline__ int row_role(const DevModel& m, int64_t i, int k) {
  if (m.fold_kind == PCV_FOLDS_INDEX) {
    const int f = m.fold_index[i];
    return f == k ? 2 : 1;
  }
  if (m.fold_kind == PCV_FOLDS_INTERVALS) {
    const int32_t* v = m.ivals + 4 * k;
    if (i >= v[0] && i < v[1]) return 2;
    if (i >= v[2] && i < v[3]) return 0;
    return 1;
  }
  return m.roles[static_cast<int64_t>(k) * m.n + i];
}

// ----------------------------------------------------------------------------
// Per-chain device routines shared by the fused and the split paths.
// State arrays are [d][C]; c is the local chain index.
// ----------------------------------------------------------------------------

// eta of row i for chain c at position q ([d][C]) in fp64.
__device__ __forceinline__ double eta_row64(const DevModel& m, const double* q, int64_t c, int64_t i) {
  const double* x = m.X64 + i * m.p;
  double e = 0.0;
  const uint8_t* mrow = mask_row(m, c);
  for (int64_t j = 0; j < m.p; ++j) e += x[j] * (covariate_used(mrow, j) ? q[j * m.C + c] : 0.0);
  if (hier_family(m.family)) {
    const double mu = q[m.p * m.C + c];
    const double tau = exp(q[(m.p + 1) * m.C + c]);
    e += mu + tau * q[(hier_z0(m) + m.group_of[i]) * m.C + c];
  }
  return e;
}

// Log density (fp64, with constants) of test slots [a0, a1) of chain c's
// fold at q; the group location and scale are read once.
template <int FAM, bool MASKED>
__device__ double log_pred_rows_m(const DevModel& m, const double* q, int64_t c, int a0, int a1) {
  double mu = 0.0, tau = 0.0, is2 = m.inv_sigma2, lsy = 0.0;
  const int64_t z0 = hier_z0(m);
  if (hier_fam<FAM>()) {
    mu = q[m.p * m.C + c];
    tau = exp(q[(m.p + 1) * m.C + c]);
  }
  if (FAM == FAM_HGAUSS) {
    lsy = q[(m.p + 2) * m.C + c];
    is2 = exp(-2.0 * lsy);
  }
  const uint8_t* mrow = MASKED ? mask_row(m, c) : nullptr;
  // coefficient j of the chain, zero where its model drops j (loads first,
  // unconditionally, then the selection: a guarded load waits alone)
  auto coef = [&](int64_t j) {
    const double v = q[j * m.C + c];
    if (!MASKED) return v;
    const uint8_t keep = mrow[j];
    return keep ? v : 0.0;
  };
  double s = 0.0;
  // Four rows at a time (a last group of two or three masked, a last single
  // row on its own), LPB coefficients per batch of loads, so that loads
  // overlap; each row's arithmetic and the order of the sum over rows are
  // those of a plain row-by-row loop.
  constexpr int LPB = 4;
  for (int t = a0; t < a1; t += 4) {
    if (t + 1 == a1) {
      const int64_t i = m.test_rows[t];
      const double* x = m.X64 + i * m.p;
      double e = 0.0;
      for (int64_t j = 0; j < m.p; ++j) e += x[j] * coef(j);
      if (hier_fam<FAM>()) e += mu + tau * q[(z0 + m.group_of[i]) * m.C + c];
      s += ell0_64<FAM>(m.y64[i], e, is2) + m.rowc[i] - lsy;
      break;
    }
    int64_t i[4];
    double e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      i[u] = m.test_rows[t + u < a1 ? t + u : t];
      e[u] = 0.0;
    }
    for (int64_t j0 = 0; j0 < m.p; j0 += LPB) {
      double qj[LPB], xv[4][LPB];
#pragma unroll
      for (int v = 0; v < LPB; ++v) {
        const int64_t j = j0 + v < m.p ? j0 + v : j0;
        qj[v] = coef(j);
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u][v] = m.X64[i[u] * m.p + j];
      }
#pragma unroll
      for (int v = 0; v < LPB; ++v)
        if (j0 + v < m.p) {
#pragma unroll
          for (int u = 0; u < 4; ++u) e[u] += xv[u][v] * qj[v];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (t + u < a1) {
        if (hier_fam<FAM>()) e[u] += mu + tau * q[(z0 + m.group_of[i[u]]) * m.C + c];
        s += ell0_64<FAM>(m.y64[i[u]], e[u], is2) + m.rowc[i[u]] - lsy;
      }
    }
  }
  return s;
}
template <int FAM>
__device__ double log_pred_rows(const DevModel& m, const double* q, int64_t c, int a0, int a1) {
  return m.mmask ? log_pred_rows_m<FAM, true>(m, q, c, a0, a1) : log_pred_rows_m<FAM, false>(m, q, c, a0, a1);
}

// Joint log density of the fold's test rows at q (fp64, with constants).
template <int FAM>
__device__ double log_pred_fold(const DevModel& m, const double* q, int64_t c) {
  const int k = fold_of_chain(m, c);
  return log_pred_rows<FAM>(m, q, c, m.test_ptr[k], m.test_ptr[k + 1]);
}

// Coordinate j's share of prior_quad at value t.
__device__ __forceinline__ double prior_term(const DevModel& m, double t, int64_t j) {
  if (m.family == FAM_HGAUSS) {
    if (j == m.p + 1 || j == m.p + 2) return -0.5 * exp(2.0 * t) / HGAUSS_SCALE_VAR + t;
    return -0.5 * t * t;
  }
  if (m.family == FAM_HIER) {
    if (j == m.p + 1) {
      const double tau = exp(t);
      return -0.5 * tau * tau + t;
    }
    return -0.5 * t * t;
  }
  return -0.5 * t * t * m.prior_prec[j];
}

// Prior: returns the non-constant part of log prior at q (constants are in
// fold_const).  For FAM_HGAUSS it also carries the likelihood's chain-dependent
// normalisation, -n_train(k) log sigma_y.
__device__ __forceinline__ double prior_quad(const DevModel& m, const double* q, int64_t c) {
  double v = 0.0;
  if (m.family == FAM_HGAUSS) {
    // beta, mu, z ~ N(0, 1); sigma_a, sigma_y half-normal (variance 10) with
    // the log-Jacobians; plus the likelihood's -n_train log sigma_y
    for (int64_t j = 0; j < m.d; ++j) v += prior_term(m, q[j * m.C + c], j);
    v -= m.ntrain[fold_of_chain(m, c)] * q[(m.p + 2) * m.C + c];
    return v;
  }
  if (m.family == FAM_HIER) {
    for (int64_t j = 0; j < m.d; ++j) {
      if (j == m.p + 1) continue;
      const double t = q[j * m.C + c];
      v -= 0.5 * t * t;
    }
    const double u = q[(m.p + 1) * m.C + c];
    const double tau = exp(u);
    v += -0.5 * tau * tau + u;
    return v;
  }
  for (int64_t j = 0; j < m.d; ++j) {
    const double t = q[j * m.C + c];
    v -= 0.5 * t * t * m.prior_prec[j];
  }
  return v;
}

__device__ __forceinline__ double prior_grad(const DevModel& m, double theta, int64_t j) {
  if (m.family == FAM_HGAUSS) {
    if (j == m.p + 1 || j == m.p + 2) return -exp(2.0 * theta) / HGAUSS_SCALE_VAR + 1.0;
    return -theta;
  }
  if (m.family == FAM_HIER) {
    if (j == m.p + 1) return -exp(2.0 * theta) + 1.0;
    return -theta;
  }
  return -theta * m.prior_prec[j];
}

// Momentum coordinates 2 jb and 2 jb + 1 of chain c at transition t (one
// Philox block, Box-Muller), their half kick and drift; adds their kinetic
// energy to k0.
__device__ __forceinline__ void momentum_pair(const DevModel& m, int64_t c, int64_t t, int64_t jb, double& k0) {
  const uint32_t gc = static_cast<uint32_t>(m.chain_offset + c);
  const W4 w = philox4x32_10(W4{gc, static_cast<uint32_t>(t), TAG_MOMENTUM, static_cast<uint32_t>(jb)},
                             m.key0, m.key1);
  const double u1 = uniform01(w.x, w.y), u2 = uniform01(w.z, w.w);
  const double r = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  const double z[2] = {r * cos(ang), r * sin(ang)};
  for (int h = 0; h < 2; ++h) {
    const int64_t j = 2 * jb + h;
    if (j >= m.d) break;
    const double mi = m.minv[j];
    double p = z[h] / sqrt(mi);
    k0 += 0.5 * mi * p * p;
    const int64_t o = j * m.C + c;
    p += 0.5 * m.eps * m.g0[o];
    m.pm[o] = p;
    m.q1[o] = m.q0[o] + m.eps * mi * p;
  }
}

// Momentum refresh, first half kick and first drift of one transition.
__device__ __forceinline__ void momentum_and_first_drift(const DevModel& m, int64_t c, int64_t t) {
  double k0 = 0.0;
  for (int64_t jb = 0; 2 * jb < m.d; ++jb) momentum_pair(m, c, t, jb, k0);
  m.h0[c] = -m.logp0[c] + k0;
}

// Leapfrog update after a gradient evaluation at q1 (g already includes the prior).
// last: half kick only; otherwise full kick and drift.
__device__ __forceinline__ void leapfrog_update(const DevModel& m, int64_t c, int64_t j, double g, bool last) {
  const int64_t o = j * m.C + c;
  m.g1[o] = g;
  double p = m.pm[o];
  if (last) {
    p += 0.5 * m.eps * g;
    m.pm[o] = p;
  } else {
    p += m.eps * g;
    m.pm[o] = p;
    m.q1[o] += m.eps * m.minv[j] * p;
  }
}

// Welford (or shifted-sum) / log-sum-exp accumulation of post-warm-up draw i
// (Algorithm A2).  The chain's accumulators are all read before any is
// written, so their loads are in flight together.
__device__ __forceinline__ void accumulate_draw(const DevModel& m, int64_t c, int64_t i, double s) {
  const int64_t per_block = static_cast<int64_t>(m.Gb) * m.b;
  int64_t blk = i / per_block;
  if (blk > m.D - 1) blk = m.D - 1;
  const double cnt = static_cast<double>(i - blk * per_block + 1);
  const int64_t o = blk * m.C + c;
  const bool batch_end = (i + 1) % m.b == 0;
  const double z0 = m.Z[c], u20 = m.U2[c], mean = m.bmean[o], m2 = m.bm2[o];
  const double ctr = m.center[c / m.L];   // read in both modes (the shifted-sums centre)
  double u0 = 0.0, v0 = 0.0, v20 = 0.0;
  if (batch_end) {
    u0 = m.U[c];
    v0 = m.V[c];
    v20 = m.V2[c];
  }
  const double z = log_add_exp(z0, s);
  m.U2[c] = log_add_exp(u20, 2.0 * s);
  if (m.rhat_mode == 1) {
    const double dv = s - ctr;
    m.bmean[o] = mean + dv;
    m.bm2[o] = m2 + dv * dv;
  } else {
    const double delta = s - mean;
    const double nm = mean + delta / cnt;
    m.bmean[o] = nm;
    m.bm2[o] = m2 + delta * (s - nm);
  }
  if (batch_end) {
    const double lb = log(static_cast<double>(m.b));
    m.U[c] = log_add_exp(u0, z);
    m.V[c] = log_add_exp(v0, z - lb);
    m.V2[c] = log_add_exp(v20, 2.0 * z - 2.0 * lb);
    m.Z[c] = -INFINITY;
  } else {
    m.Z[c] = z;
  }
}

// One predictive draw of y given eta from the Philox block w: Gaussian by
// Box-Muller, Bernoulli by threshold, Poisson by inverse cdf.
template <int FAM>
__device__ double predictive_draw(const DevModel& m, double eta, W4 w) {
  const double u = uniform01(w.x, w.y);
  if (FAM == FAM_GAUSS) {
    const double u2 = uniform01(w.z, w.w);
    return eta + m.sigma * sqrt(-2.0 * log(u)) * cos(2.0 * M_PI * u2);
  }
  if (FAM == FAM_LOGIT || FAM == FAM_HIER) return u < 1.0 / (1.0 + exp(-eta)) ? 1.0 : 0.0;
  const double lam = exp(eta);
  double p = exp(-lam), F = p, k = 0.0;
  for (int j = 1; u > F && j <= 100000; ++j) {
    p = p * lam / j;
    F += p;
    k += 1.0;
  }
  return k;
}

// HS and DSS sums of one post-warm-up draw at the accepted state q0.
template <int FAM>
__device__ void accumulate_scores(const DevModel& m, int64_t c, int64_t t) {
  if (FAM == FAM_HGAUSS) return;   // pcv_init refuses HS / DSS for this family
  const int k = fold_of_chain(m, c);
  const int64_t l = c % m.L;
  const int beg = m.test_ptr[k], v = m.test_ptr[k + 1] - beg;
  const int64_t o1 = static_cast<int64_t>(m.L) * beg + l * v;
  const uint32_t gc = static_cast<uint32_t>(m.chain_offset + c);
  double h1 = 0.0;
  for (int a = 0; a < v; ++a) {
    const int64_t i = m.test_rows[beg + a];
    const double eta = eta_row64(m, m.q0, c, i);
    const double y = m.y64[i];
    if (m.scores & 1) {
      const double d1 = -(y - eta) * m.inv_sigma2;
      h1 += -m.inv_sigma2 + d1 * d1;
      m.hs2[o1 + a] += d1;
    }
    if (m.scores & 2) {
      const W4 w = philox4x32_10(W4{gc, static_cast<uint32_t>(t), TAG_PREDICT, static_cast<uint32_t>(a)}, m.key0,
                                 m.key1);
      const double r = predictive_draw<FAM>(m, eta, w) - y;
      m.dx[o1 + a] += r;
      m.rcur[o1 + a] = r;
    }
  }
  if (m.scores & 1) m.hs1[c] += h1;
  if (m.scores & 2) {
    const int64_t o2 = static_cast<int64_t>(m.L) * m.sq_ptr[k] + l * v * v;
    for (int a = 0; a < v; ++a) {
      const double ra = m.rcur[o1 + a];
      for (int b = 0; b < v; ++b) m.dxx[o2 + static_cast<int64_t>(a) * v + b] += ra * m.rcur[o1 + b];
    }
  }
}

// Metropolis test of chain c at transition t, given log pi and the kinetic
// energy k1 at the end of its trajectory.
__device__ __forceinline__ void metropolis(const DevModel& m, int64_t c, int64_t t, double logp1, double k1,
                                           bool& accepted, bool& divergent) {
  const double h1 = -logp1 + k1;
  const double log_ratio = m.h0[c] - h1;
  const uint32_t gc = static_cast<uint32_t>(m.chain_offset + c);
  const W4 w = philox4x32_10(W4{gc, static_cast<uint32_t>(t), TAG_ACCEPT, 0u}, m.key0, m.key1);
  const double u = uniform01(w.x, w.y);
  const bool finite = isfinite(log_ratio);
  accepted = finite && (log(u) < log_ratio);
  divergent = !finite || (-log_ratio > DIVERGENCE_THRESHOLD);
  if (m.acc_stat) m.acc_stat[c] = finite ? (log_ratio >= 0.0 ? 1.0 : exp(log_ratio)) : 0.0;
}

// Bookkeeping of transition t once the state (q0, s0) is selected: warm-up
// sums, or the online accumulators, scores, stored draw and counters.
template <int FAM>
// s0 is the log predictive of the selected state (the value s0[c] holds).
__device__ void record_draw(const DevModel& m, int64_t c, int64_t t, bool accepted, bool divergent, double s0) {
  if (t < m.n_warmup) {
    if (m.rhat_mode == 1) m.wsum[c] += s0;
  } else {
    const int64_t na = m.nacc[c], nd = m.ndiv[c];   // read before the accumulators are written
    accumulate_draw(m, c, t - m.n_warmup, s0);
    if (m.scores) accumulate_scores<FAM>(m, c, t);
    const int64_t di = t - m.n_warmup;
    if (m.draws && di < m.draws_cap) m.draws[di * m.C + c] = s0;
    m.nacc[c] = na + (accepted ? 1 : 0);
    m.ndiv[c] = nd + (divergent ? 1 : 0);
  }
}

// Metropolis test at the end of a trajectory (q1, pm, logp1, g1), state
// selection, log predictive at the new state and accumulation.
template <int FAM>
__device__ void accept_and_accumulate(const DevModel& m, int64_t c, int64_t t) {
  double k1 = 0.0;
  for (int64_t j = 0; j < m.d; ++j) {
    const double p = m.pm[j * m.C + c];
    k1 += 0.5 * m.minv[j] * p * p;
  }
  bool accepted, divergent;
  metropolis(m, c, t, m.logp1[c], k1, accepted, divergent);
  double s0;
  if (accepted) {
    for (int64_t j = 0; j < m.d; ++j) {
      const int64_t o = j * m.C + c;
      m.q0[o] = m.q1[o];
      m.g0[o] = m.g1[o];
    }
    m.logp0[c] = m.logp1[c];
    s0 = log_pred_fold<FAM>(m, m.q0, c);
    m.s0[c] = s0;
  } else {
    s0 = m.s0[c];
  }
  record_draw<FAM>(m, c, t, accepted, divergent, s0);
}

}  // namespace pcv
