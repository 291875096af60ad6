// Per-chain kernels of the split (multi-launch) paths, diagnostics, and
// initialisation helpers.
#include "pcv_internal.h"

namespace pcv {

constexpr int TPB = 256;

static inline int nblocks(int64_t n, int tpb = TPB) { return static_cast<int>((n + tpb - 1) / tpb); }

// ---- transition pieces -----------------------------------------------------

// Advance the device-side transition counter (last node of a captured transition).
__global__ void k_tick(DevModel m) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *m.t_dev += 1;
}

// Sum partial gradients over row splits (fixed order), add the prior, and
// apply the leapfrog update.  mode 0: store the gradient only; 1: kick and
// drift; 2: final half kick.
template <typename PT>
__global__ void k_reduce(DevModel m, const PT* __restrict__ Gpart, int n_splits, int mode) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= m.d * m.C) return;
  const int64_t j = idx / m.C, c = idx - j * m.C;
  // loads issued sixteen at a time, added in split order
  const PT* gp = Gpart + idx;
  const int64_t dC = m.d * m.C;
  double G = 0.0;
  int s = 0;
  for (; s + 16 <= n_splits; s += 16) {
    PT t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = gp[(s + u) * dC];
#pragma unroll
    for (int u = 0; u < 16; ++u) G += static_cast<double>(t[u]);
  }
  if (s + 8 <= n_splits) {
    PT t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = gp[(s + u) * dC];
#pragma unroll
    for (int u = 0; u < 8; ++u) G += static_cast<double>(t[u]);
    s += 8;
  }
  for (; s < n_splits; ++s) G += static_cast<double>(gp[s * dC]);
  if (!covariate_used(mask_row(m, c), j)) G = 0.0;   // a masked coefficient: prior only
  const double g = G + prior_grad(m, m.q1[idx], j);
  if (mode == 0) m.g1[idx] = g;
  else leapfrog_update(m, c, j, g, mode == 2);
}

__device__ __forceinline__ double value_finish(const DevModel& m, const double* Vpart, int n_splits, int64_t c) {
  double v = 0.0;
  for (int s = 0; s < n_splits; ++s) v += Vpart[static_cast<int64_t>(s) * m.C + c];
  return v + m.fold_const[fold_of_chain(m, c)] + prior_quad(m, m.q1, c);
}

__global__ void k_value_finish(DevModel m, const double* Vpart, int n_splits) {
  const int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (c < m.C) m.logp1[c] = value_finish(m, Vpart, n_splits, c);
}

// ---- block-wide transition pieces of the split paths -------------------------
// One workgroup per 64 chains (lane = chain); its Y waves share each chain's
// loops over coordinates, value partials and test rows, and the per-wave
// partial sums are added in a fixed order (bit-reproducible).

constexpr int WIDE_MAX_Y = 16;

// Momentum refresh, first half kick and drift; the waves take the Philox
// blocks jb = y, y + Y, ...
__global__ __launch_bounds__(64 * WIDE_MAX_Y) void k_momentum(DevModel m, int64_t t) {
  __shared__ double red[WIDE_MAX_Y][64];
  const int lane = threadIdx.x & 63, y = threadIdx.x >> 6, Y = blockDim.x >> 6;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  const bool valid = c < m.C;
  if (t < 0) t = *m.t_dev;
  double k0 = 0.0;
  if (valid)
    for (int64_t jb = y; 2 * jb < m.d; jb += Y) momentum_pair(m, c, t, jb, k0);
  red[y][lane] = k0;
  __syncthreads();
  if (y == 0 && valid) {
    double s = 0.0;
    for (int w = 0; w < Y; ++w) s += red[w][lane];
    m.h0[c] = -m.logp0[c] + s;
  }
}

// Metropolis test and accumulation.  Phase 1 (all waves): value partials,
// prior, kinetic energy and the log predictive of the proposal q1 (the
// partial sums k_testlp wrote, or a contiguous share of the fold's test
// rows evaluated here).  Phase 2 (wave 0): log pi(q1),
// the test, logp0 and s0 (the proposal's log predictive when accepted).
// Phase 3 (all waves): q0, g0 := q1, g1 for accepted chains.  Phase 4
// (wave 0): accumulation, which reads the selected q0 for the scores.
// Waves per workgroup of k_accept: the Gaussian family's score draws need
// the registers of 512-thread groups; the others fit 1024-thread groups.
template <int FAM>
constexpr int accept_max_y() { return FAM == FAM_GAUSS ? 8 : WIDE_MAX_Y; }

template <int FAM>
__global__ __launch_bounds__(64 * accept_max_y<FAM>()) void k_accept(DevModel m, const double* __restrict__ Vpart,
                                                                     int n_splits, int64_t t) {
  __shared__ double red[4][accept_max_y<FAM>()][64];
  __shared__ int acc_s[64];
  const int lane = threadIdx.x & 63, y = threadIdx.x >> 6, Y = blockDim.x >> 6;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + lane;
  const bool valid = c < m.C;
  const int64_t cc = valid ? c : m.C - 1;
  if (t < 0) t = *m.t_dev;
  double v = 0.0, pq = 0.0, k1 = 0.0, lp = 0.0;
  for (int s = y; s < n_splits; s += Y) v += Vpart[static_cast<int64_t>(s) * m.C + cc];
  // coordinates y, y + Y, ... in batches of four: loads from clamped indices
  // first (all in flight), then the sums in coordinate order
  for (int64_t j0 = y; j0 < m.d; j0 += 4 * Y) {
    double qv[4], pv[4], mv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + u * Y < m.d ? j0 + u * Y : j0;
      const int64_t o = j * m.C + cc;
      qv[u] = m.q1[o];
      pv[u] = m.pm[o];
      mv[u] = m.minv[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + u * Y < m.d) {
        pq += prior_term(m, qv[u], j0 + u * Y);
        k1 += 0.5 * mv[u] * pv[u] * pv[u];
      }
  }
  const int k = fold_of_chain(m, cc);
  // the hierarchical Gaussian's -n_train log sigma_y (prior_quad's extra term)
  if (FAM == FAM_HGAUSS && y == 0) pq -= m.ntrain[k] * m.q1[(m.p + 2) * m.C + cc];
  // the proposal's log predictive: k_testlp's partial sums, or (folds with
  // few test rows) this wave's contiguous share of the fold's test rows
  if (m.lp_part) {
    for (int g = y; g < m.lp_groups; g += Y) lp += m.lp_part[static_cast<int64_t>(g) * m.C + cc];
  } else {
    const int beg = m.test_ptr[k], nt = m.test_ptr[k + 1] - beg;
    lp = log_pred_rows<FAM>(m, m.q1, cc, beg + static_cast<int>(static_cast<int64_t>(nt) * y / Y),
                            beg + static_cast<int>(static_cast<int64_t>(nt) * (y + 1) / Y));
  }
  red[0][y][lane] = v;
  red[1][y][lane] = pq;
  red[2][y][lane] = k1;
  red[3][y][lane] = lp;
  __syncthreads();
  bool accepted = false, divergent = false;
  double s_sel = 0.0;   // log predictive of the selected state (wave 0)
  if (y == 0) {
    const double s_prev = m.s0[cc];
    v = pq = k1 = lp = 0.0;
    for (int w = 0; w < Y; ++w) {
      v += red[0][w][lane];
      pq += red[1][w][lane];
      k1 += red[2][w][lane];
      lp += red[3][w][lane];
    }
    if (valid) {
      const double logp1 = v + m.fold_const[k] + pq;
      m.logp1[c] = logp1;
      metropolis(m, c, t, logp1, k1, accepted, divergent);
      if (accepted) {
        m.logp0[c] = logp1;
        m.s0[c] = lp;
      }
      s_sel = accepted ? lp : s_prev;
    }
    acc_s[lane] = accepted ? 1 : 0;
  }
  __syncthreads();
  if (valid && acc_s[lane]) {
    // batches of four coordinates: loads first, then the stores
    for (int64_t j0 = y; j0 < m.d; j0 += 4 * Y) {
      double qv[4], gv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + u * Y < m.d ? j0 + u * Y : j0;
        qv[u] = m.q1[j * m.C + c];
        gv[u] = m.g1[j * m.C + c];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u * Y < m.d) {
          m.q0[(j0 + u * Y) * m.C + c] = qv[u];
          m.g0[(j0 + u * Y) * m.C + c] = gv[u];
        }
    }
  }
  __syncthreads();
  if (y == 0 && valid) record_draw<FAM>(m, c, t, accepted, divergent, s_sel);
}

// Log predictive of the proposal q1 over each chain's test rows (eq cv-score's
// log p(y_test | theta)), spread over the chip for k_accept: workgroup
// (chain block, group g) with Y waves; wave w takes test slot a = g Y + w of
// each lane's fold (one row: eta summed over the coefficients in order, then
// the row's log density with its constant), and the waves' terms are added in
// wave order into lp_part[g][c].  The block's coefficients (zero where a
// nested model drops one) are staged in LDS once, so the Y waves read them
// there instead of each fetching all of them again from L2.
constexpr int TESTLP_MAX_P = 128;
template <int FAM, bool MASKED>
__global__ __launch_bounds__(64 * WIDE_MAX_Y) void k_testlp(DevModel m) {
  __shared__ double sq[TESTLP_MAX_P * 64];   // [j][lane]
  __shared__ double red[WIDE_MAX_Y][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, Y = blockDim.x >> 6;
  const int64_t cbase = static_cast<int64_t>(blockIdx.x) * 64;
  const int p = static_cast<int>(m.p);
  for (int t = threadIdx.x; t < p * 64; t += blockDim.x) {
    const int j = t >> 6, l = t & 63;
    const int64_t cl = cbase + l < m.C ? cbase + l : m.C - 1;
    const double v = m.q1[static_cast<int64_t>(j) * m.C + cl];
    if (MASKED) {
      const uint8_t keep = mask_row(m, cl)[j];
      sq[t] = keep ? v : 0.0;
    } else {
      sq[t] = v;
    }
  }
  __syncthreads();
  const int64_t c = cbase + lane;
  const bool valid = c < m.C;
  const int64_t cc = valid ? c : m.C - 1;
  const int k = fold_of_chain(m, cc);
  const int beg = m.test_ptr[k], nt = m.test_ptr[k + 1] - beg;
  const int a = static_cast<int>(blockIdx.y) * Y + w;
  double s = 0.0;
  if (a < nt) {
    const int64_t i = m.test_rows[beg + a];
    const double* x = m.X64 + i * m.p;
    double e = 0.0;
    constexpr int LB = 16;
    for (int j0 = 0; j0 < p; j0 += LB) {
      double xv[LB];
#pragma unroll
      for (int v = 0; v < LB; ++v) xv[v] = x[j0 + v < p ? j0 + v : j0];
#pragma unroll
      for (int v = 0; v < LB; ++v)
        if (j0 + v < p) e += xv[v] * sq[(j0 + v) * 64 + lane];
    }
    double is2 = m.inv_sigma2, lsy = 0.0;
    if (hier_fam<FAM>())
      e += m.q1[m.p * m.C + cc] + exp(m.q1[(m.p + 1) * m.C + cc]) * m.q1[(hier_z0(m) + m.group_of[i]) * m.C + cc];
    if (FAM == FAM_HGAUSS) {
      lsy = m.q1[(m.p + 2) * m.C + cc];
      is2 = exp(-2.0 * lsy);
    }
    s = ell0_64<FAM>(m.y64[i], e, is2) + m.rowc[i] - lsy;
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && valid) {
    double v = 0.0;
    for (int u = 0; u < Y; ++u) v += red[u][lane];
    m.lp_part[static_cast<int64_t>(blockIdx.y) * m.C + c] = v;
  }
}

// Log predictive at q0 for every chain (initialisation and set_state).
template <int FAM>
__global__ void k_logpred(DevModel m) {
  const int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (c < m.C) m.s0[c] = log_pred_fold<FAM>(m, m.q0, c);
}

// Masked residual of the unfused fp64 path, eta [n][cc] column-major (one
// column per chain), in place; one block per chain column; value partial.
template <int FAM>
__global__ void k_unfused_resid(DevModel m, double* __restrict__ eta, int64_t c0, int64_t cc, double* Vpart,
                                int want_value) {
  __shared__ double red[TPB];
  const int64_t col = blockIdx.x;
  if (col >= cc) return;
  const int64_t c = c0 + col;
  const int k = fold_of_chain(m, c);
  double v = 0.0;
  double* e = eta + col * m.n;
  for (int64_t i = threadIdx.x; i < m.n; i += blockDim.x) {
    const bool train = row_role(m, i, k) == 1;
    const double et = e[i];
    const double y = m.y64[i];
    if (want_value && train) v += ell0_64<FAM>(y, et, m.inv_sigma2);
    e[i] = train ? resid64<FAM>(y, et, m.inv_sigma2) : 0.0;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && want_value) Vpart[c] = red[0];
}

// ---- initialisation helpers ------------------------------------------------

__global__ void k_rowconst(DevModel m, double* rowc) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= m.n) return;
  double v = 0.0;
  if (m.family == FAM_GAUSS) v = -0.5 * log(2.0 * M_PI / m.inv_sigma2);
  else if (m.family == FAM_HGAUSS) v = -0.5 * log(2.0 * M_PI);   // -log sigma_y is per chain
  else if (m.family == FAM_POIS) v = -lgamma(m.y64[i] + 1.0);
  rowc[i] = v;
}

// fold_const[k] = sum over train rows of the row constant + prior constant.
__global__ void k_foldconst(DevModel m, double prior_const, double* fold_const) {
  __shared__ double red[TPB];
  const int k = blockIdx.x;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < m.n; i += blockDim.x)
    if (row_role(m, i, k) == 1) v += m.rowc[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) fold_const[k] = red[0] + prior_const;
}

// [C][d] chain-major <-> [d][C]
__global__ void k_to_dc(const double* __restrict__ src, double* __restrict__ dst, int64_t C, int64_t d) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= C * d) return;
  const int64_t j = idx / C, c = idx - j * C;
  dst[idx] = src[c * d + j];
}
__global__ void k_to_cd(const double* __restrict__ src, double* __restrict__ dst, int64_t C, int64_t d) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= C * d) return;
  const int64_t c = idx / d, j = idx - c * d;
  dst[idx] = src[j * C + c];
}

__global__ void k_fill(double* p, double v, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                         uint32_t* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const W4 w = philox4x32_10(W4{c0, c1, c2, c3 + static_cast<uint32_t>(i)}, k0, k1);
  out[4 * i + 0] = w.x;
  out[4 * i + 1] = w.y;
  out[4 * i + 2] = w.z;
  out[4 * i + 3] = w.w;
}

// ---- diagnostics (fp64) ----------------------------------------------------
// Per fold: elpd_k, Rhat_k, sigma2_k/f_k^2 (batch means), s2_k/f_k^2 (pooled),
// ESS_k, Var(f_k)/f_k^2.  Every exponential is taken relative to the fold's
// largest log term.
struct FoldDiag {
  double* elpd;
  double* rhat;
  double* sig2rel;
  double* s2rel;
  double* ess;
  double* varrel;
};

__device__ __forceinline__ void chan_merge(double& n, double& mean, double& m2, double nb, double mb, double m2b) {
  const double nt = n + nb;
  if (nt <= 0.0) return;
  const double delta = mb - mean;
  mean = mean + delta * (nb / nt);
  m2 = m2 + m2b + delta * delta * n * nb / nt;
  n = nt;
}

// Combine block statistics into a chain's.  Welford blocks (count, mean, M2)
// Chan-merge.  Shifted-sum blocks (count, Y = sum (s - C_k), Y2 = sum
// (s - C_k)^2) add, and block_finish turns the totals into the mean of
// s - C_k and M2 = Y2 - Y^2 / n (the shift drops out of Rhat).
__device__ __forceinline__ void block_merge(const DevModel& m, double& n, double& a, double& b, double nb,
                                            double ab, double bb) {
  if (m.rhat_mode == 1) {
    n += nb;
    a += ab;
    b += bb;
  } else {
    chan_merge(n, a, b, nb, ab, bb);
  }
}
__device__ __forceinline__ void block_finish(const DevModel& m, double n, double& a, double& b) {
  if (m.rhat_mode == 1 && n > 0.0) {
    const double y = a;
    a = y / n;
    b = b - y * y / n;
  }
}

__device__ __forceinline__ double block_count(const DevModel& m, int64_t N, int dd) {
  const int64_t per = static_cast<int64_t>(m.Gb) * m.b;
  int64_t lo = dd * per, hi = (dd == m.D - 1) ? N : (dd + 1) * per;
  if (hi > N) hi = N;
  return hi > lo ? static_cast<double>(hi - lo) : 0.0;
}

__device__ double rhat_of(double N, const double* mean, const double* m2, int L) {
  double W = 0.0, grand = 0.0;
  for (int l = 0; l < L; ++l) {
    W += m2[l] / (N - 1.0);
    grand += mean[l];
  }
  W /= L;
  grand /= L;
  double B = 0.0;
  for (int l = 0; l < L; ++l) B += (mean[l] - grand) * (mean[l] - grand);
  B *= N / (L - 1.0);
  return sqrt((N - 1.0) / N + B / (N * W));
}

constexpr int MAX_L = 64;

__global__ void k_diag_fold(DevModel m, int64_t N, FoldDiag o) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.K) return;
  const int L = m.L;
  const int64_t c0 = static_cast<int64_t>(k) * L;
  const double LN = static_cast<double>(L) * N;
  // elpd and pooled variance of f = e^s
  double ua[MAX_L];
  double mu = -INFINITY;
  for (int l = 0; l < L; ++l) {
    ua[l] = log_add_exp(m.U[c0 + l], m.Z[c0 + l]);
    mu = fmax(mu, ua[l]);
  }
  double s1 = 0.0, s2 = 0.0;
  for (int l = 0; l < L; ++l) {
    s1 += exp(ua[l] - mu);
    s2 += exp(m.U2[c0 + l] - 2.0 * mu);
  }
  const double log_fhat = mu + log(s1) - log(LN);
  o.elpd[k] = log_fhat;
  const double br = s2 - s1 * s1 / LN;
  const double s2rel = exp(2.0 * mu + log(fmax(br, 0.0)) - log(LN - 1.0) - 2.0 * log_fhat);
  o.s2rel[k] = s2rel;
  // batch means
  const int64_t a = N / m.b;
  double sig2rel = NAN;
  if (a >= 1 && L * a > 1) {
    double mv = -INFINITY;
    for (int l = 0; l < L; ++l) mv = fmax(mv, m.V[c0 + l]);
    double v1 = 0.0, v2 = 0.0;
    for (int l = 0; l < L; ++l) {
      v1 += exp(m.V[c0 + l] - mv);
      v2 += exp(m.V2[c0 + l] - 2.0 * mv);
    }
    const double La = static_cast<double>(L) * a;
    const double bv = v2 - v1 * v1 / La;
    sig2rel = exp(log(static_cast<double>(m.b)) - log(La - 1.0) + 2.0 * mv + log(fmax(bv, 0.0)) - 2.0 * log_fhat);
  }
  o.sig2rel[k] = sig2rel;
  o.varrel[k] = sig2rel / LN;
  o.ess[k] = LN * s2rel / sig2rel;
  // Rhat from the blocks of each chain
  double cm[MAX_L], cm2[MAX_L];
  for (int l = 0; l < L; ++l) {
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int dd = 0; dd < m.D; ++dd) {
      const int64_t off = static_cast<int64_t>(dd) * m.C + c0 + l;
      block_merge(m, n, mean, m2, block_count(m, N, dd), m.bmean[off], m.bm2[off]);
    }
    block_finish(m, n, mean, m2);
    cm[l] = mean;
    cm2[l] = m2;
  }
  o.rhat[k] = N >= 2 ? rhat_of(static_cast<double>(N), cm, cm2, L) : NAN;
}

// Fold-level sums and max, one block, fixed-order tree (deterministic).
// out: [0] sum elpd, [1] max rhat, [2] sum varrel, [3] sum s2rel, [4] sum sig2rel
__global__ void k_diag_reduce(int K, FoldDiag o, double* out) {
  __shared__ double r[5][1024];
  double a0 = 0.0, a1 = -INFINITY, a2 = 0.0, a3 = 0.0, a4 = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    a0 += o.elpd[k];
    a1 = fmax(a1, o.rhat[k]);
    a2 += o.varrel[k];
    a3 += o.s2rel[k];
    a4 += o.sig2rel[k];
  }
  r[0][threadIdx.x] = a0;
  r[1][threadIdx.x] = a1;
  r[2][threadIdx.x] = a2;
  r[3][threadIdx.x] = a3;
  r[4][threadIdx.x] = a4;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      r[0][threadIdx.x] += r[0][threadIdx.x + s];
      r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + s]);
      r[2][threadIdx.x] += r[2][threadIdx.x + s];
      r[3][threadIdx.x] += r[3][threadIdx.x + s];
      r[4][threadIdx.x] += r[4][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 5; ++q) out[q] = r[q][0];
}

// Block-shuffle replicate r of fold k (Section 4.2): chain slot l takes block
// dd from chain floor(u * L) of the same fold, u from Philox(fold, r, TAG, l*D+dd).
__global__ void k_shuffle(DevModel m, int64_t N, int R, uint32_t s0, uint32_t s1, double* rep) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(m.K) * R) return;
  const int k = static_cast<int>(idx / R), r = static_cast<int>(idx - static_cast<int64_t>(k) * R);
  const int L = m.L;
  const uint32_t fold_global = static_cast<uint32_t>(m.chain_offset / L + k);
  double cm[MAX_L], cm2[MAX_L];
  for (int l = 0; l < L; ++l) {
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int dd = 0; dd < m.D; ++dd) {
      const W4 w = philox4x32_10(W4{fold_global, static_cast<uint32_t>(r), TAG_SHUFFLE,
                                    static_cast<uint32_t>(l * m.D + dd)}, s0, s1);
      int src = static_cast<int>(floor(uniform01(w.x, w.y) * L));
      if (src > L - 1) src = L - 1;
      const int64_t off = static_cast<int64_t>(dd) * m.C + static_cast<int64_t>(k) * L + src;
      block_merge(m, n, mean, m2, block_count(m, N, dd), m.bmean[off], m.bm2[off]);
    }
    block_finish(m, n, mean, m2);
    cm[l] = mean;
    cm2[l] = m2;
  }
  rep[idx] = rhat_of(static_cast<double>(N), cm, cm2, L);
}

// Shifted sums, end of warm-up: C_k = (sum over the fold's chains of their
// warm-up sums of s) / (L * N_wu).
__global__ void k_center(DevModel m) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.K) return;
  double t = 0.0;
  for (int l = 0; l < m.L; ++l) t += m.wsum[static_cast<int64_t>(k) * m.L + l];
  m.center[k] = m.n_warmup > 0 ? t / (static_cast<double>(m.L) * static_cast<double>(m.n_warmup)) : 0.0;
}

__global__ void k_shuffle_max(int K, int R, const double* rep, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double v = -INFINITY;
  for (int k = 0; k < K; ++k) v = fmax(v, rep[static_cast<int64_t>(k) * R + r]);
  out[r] = v;
}

// First half kick and drift from (q1, pm) with the gradient g1 at q1 (leapfrog hook).
__global__ void k_kick_drift(DevModel m) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= m.d * m.C) return;
  const int64_t j = idx / m.C;
  const double p = m.pm[idx] + 0.5 * m.eps * m.g1[idx];
  m.pm[idx] = p;
  m.q1[idx] += m.eps * m.minv[j] * p;
}

// ---- host launchers --------------------------------------------------------

#define PCV_FAM_DISPATCH(fam, KERNEL, grid, block, st, ...)                                       \
  do {                                                                                           \
    switch (fam) {                                                                               \
      case FAM_GAUSS: hipLaunchKernelGGL((KERNEL<FAM_GAUSS>), grid, block, 0, st, __VA_ARGS__); break; \
      case FAM_LOGIT: hipLaunchKernelGGL((KERNEL<FAM_LOGIT>), grid, block, 0, st, __VA_ARGS__); break; \
      case FAM_POIS: hipLaunchKernelGGL((KERNEL<FAM_POIS>), grid, block, 0, st, __VA_ARGS__); break;   \
      case FAM_HIER: hipLaunchKernelGGL((KERNEL<FAM_HIER>), grid, block, 0, st, __VA_ARGS__); break;   \
      case FAM_HGAUSS: hipLaunchKernelGGL((KERNEL<FAM_HGAUSS>), grid, block, 0, st, __VA_ARGS__); break; \
    }                                                                                            \
  } while (0)

#define PCV_FAM_DISPATCH_M(fam, KERNEL, MB, grid, block, st, ...)                                  \
  do {                                                                                           \
    switch (fam) {                                                                               \
      case FAM_GAUSS: hipLaunchKernelGGL((KERNEL<FAM_GAUSS, MB>), grid, block, 0, st, __VA_ARGS__); break; \
      case FAM_LOGIT: hipLaunchKernelGGL((KERNEL<FAM_LOGIT, MB>), grid, block, 0, st, __VA_ARGS__); break; \
      case FAM_POIS: hipLaunchKernelGGL((KERNEL<FAM_POIS, MB>), grid, block, 0, st, __VA_ARGS__); break;   \
      case FAM_HIER: hipLaunchKernelGGL((KERNEL<FAM_HIER, MB>), grid, block, 0, st, __VA_ARGS__); break;   \
      case FAM_HGAUSS: hipLaunchKernelGGL((KERNEL<FAM_HGAUSS, MB>), grid, block, 0, st, __VA_ARGS__); break; \
    }                                                                                            \
  } while (0)

hipError_t launch_tick(const DevModel& m, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, m);
  return hipGetLastError();
}
hipError_t launch_kick_drift(const DevModel& m, hipStream_t st) {
  hipLaunchKernelGGL(k_kick_drift, dim3(nblocks(m.d * m.C)), dim3(TPB), 0, st, m);
  return hipGetLastError();
}
hipError_t launch_reduce_f32(const DevModel& m, const float* G, int ns, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce<float>, dim3(nblocks(m.d * m.C)), dim3(TPB), 0, st, m, G, ns, mode);
  return hipGetLastError();
}
hipError_t launch_reduce_f64(const DevModel& m, const double* G, int ns, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce<double>, dim3(nblocks(m.d * m.C)), dim3(TPB), 0, st, m, G, ns, mode);
  return hipGetLastError();
}
hipError_t launch_value_finish(const DevModel& m, const double* V, int ns, hipStream_t st) {
  hipLaunchKernelGGL(k_value_finish, dim3(nblocks(m.C)), dim3(TPB), 0, st, m, V, ns);
  return hipGetLastError();
}
// Waves per workgroup of the block-wide kernels: enough waves to cover the
// chips' SIMDs when the chains are few.
int wide_waves(int64_t C) {
  const int64_t blocks = (C + 63) / 64;
  if (blocks < 64) return WIDE_MAX_Y;
  if (blocks < 256) return 8;
  return 4;
}
hipError_t launch_momentum(const DevModel& m, int64_t t, hipStream_t st) {
  const int Y = wide_waves(m.C);
  hipLaunchKernelGGL(k_momentum, dim3(nblocks(m.C, 64)), dim3(64 * Y), 0, st, m, t);
  return hipGetLastError();
}
hipError_t launch_accept(const DevModel& m, const double* V, int ns, int64_t t, hipStream_t st) {
  const int Y = std::min(wide_waves(m.C), m.family == FAM_GAUSS ? accept_max_y<FAM_GAUSS>() : WIDE_MAX_Y);
  PCV_FAM_DISPATCH(m.family, k_accept, dim3(nblocks(m.C, 64)), dim3(64 * Y), st, m, V, ns, t);
  return hipGetLastError();
}
// Waves per workgroup of k_testlp: one per test slot, up to WIDE_MAX_Y; the
// groups cover the largest fold's test rows.
int testlp_waves(int max_test_rows) { return std::max(1, std::min(WIDE_MAX_Y, max_test_rows)); }
int testlp_groups(int max_test_rows) {
  const int Y = testlp_waves(max_test_rows);
  return std::max(1, (max_test_rows + Y - 1) / Y);
}
hipError_t launch_testlp(const DevModel& m, int max_test_rows, hipStream_t st) {
  const dim3 grid(nblocks(m.C, 64), m.lp_groups), block(64 * testlp_waves(max_test_rows));
  if (m.mmask) PCV_FAM_DISPATCH_M(m.family, k_testlp, true, grid, block, st, m);
  else PCV_FAM_DISPATCH_M(m.family, k_testlp, false, grid, block, st, m);
  return hipGetLastError();
}
hipError_t launch_logpred(const DevModel& m, hipStream_t st) {
  PCV_FAM_DISPATCH(m.family, k_logpred, dim3(nblocks(m.C)), dim3(TPB), st, m);
  return hipGetLastError();
}
hipError_t launch_unfused_resid(const DevModel& m, double* eta, int64_t c0, int64_t cc, double* V, int want_value,
                                hipStream_t st) {
  PCV_FAM_DISPATCH(m.family, k_unfused_resid, dim3(static_cast<unsigned>(cc)), dim3(TPB), st, m, eta, c0, cc, V,
                   want_value);
  return hipGetLastError();
}
hipError_t launch_rowconst(const DevModel& m, double* rowc, hipStream_t st) {
  hipLaunchKernelGGL(k_rowconst, dim3(nblocks(m.n)), dim3(TPB), 0, st, m, rowc);
  return hipGetLastError();
}
hipError_t launch_foldconst(const DevModel& m, double prior_const, double* fc, hipStream_t st) {
  hipLaunchKernelGGL(k_foldconst, dim3(m.K), dim3(TPB), 0, st, m, prior_const, fc);
  return hipGetLastError();
}
hipError_t launch_to_dc(const double* src, double* dst, int64_t C, int64_t d, hipStream_t st) {
  hipLaunchKernelGGL(k_to_dc, dim3(nblocks(C * d)), dim3(TPB), 0, st, src, dst, C, d);
  return hipGetLastError();
}
hipError_t launch_to_cd(const double* src, double* dst, int64_t C, int64_t d, hipStream_t st) {
  hipLaunchKernelGGL(k_to_cd, dim3(nblocks(C * d)), dim3(TPB), 0, st, src, dst, C, d);
  return hipGetLastError();
}
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(TPB), 0, st, p, v, n);
  return hipGetLastError();
}
hipError_t launch_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                         uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_philox, dim3(nblocks(n)), dim3(TPB), 0, st, k0, k1, c0, c1, c2, c3, n, out);
  return hipGetLastError();
}
// The accumulator-only kernels below (centres, diagnostics, block shuffles)
// see every posterior as a fold: with several models in one launch, K
// becomes models x folds (chains k*L .. k*L + L - 1 of posterior k).
static DevModel posterior_view(const DevModel& m) {
  DevModel v = m;
  v.K = m.KP;
  return v;
}

hipError_t launch_center(const DevModel& md, hipStream_t st) {
  const DevModel m = posterior_view(md);
  hipLaunchKernelGGL(k_center, dim3(nblocks(m.K, 64)), dim3(64), 0, st, m);
  return hipGetLastError();
}

hipError_t launch_diag(const DevModel& md, int64_t N, double* fold_buf, double* out, hipStream_t st) {
  const DevModel m = posterior_view(md);
  FoldDiag o;
  o.elpd = fold_buf;
  o.rhat = fold_buf + m.K;
  o.sig2rel = fold_buf + 2 * static_cast<int64_t>(m.K);
  o.s2rel = fold_buf + 3 * static_cast<int64_t>(m.K);
  o.ess = fold_buf + 4 * static_cast<int64_t>(m.K);
  o.varrel = fold_buf + 5 * static_cast<int64_t>(m.K);
  hipLaunchKernelGGL(k_diag_fold, dim3(nblocks(m.K, 64)), dim3(64), 0, st, m, N, o);
  hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(1024), 0, st, m.K, o, out);
  return hipGetLastError();
}
hipError_t launch_shuffle(const DevModel& md, int64_t N, int R, uint32_t s0, uint32_t s1, double* rep,
                          double* repmax, hipStream_t st) {
  const DevModel m = posterior_view(md);
  hipLaunchKernelGGL(k_shuffle, dim3(nblocks(static_cast<int64_t>(m.K) * R)), dim3(TPB), 0, st, m, N, R, s0, s1,
                     rep);
  hipLaunchKernelGGL(k_shuffle_max, dim3(nblocks(R)), dim3(TPB), 0, st, m.K, R, rep, repmax);
  return hipGetLastError();
}

}  // namespace pcv
