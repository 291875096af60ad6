/* Plain C fp64 oracle of the PCV hot path: every fold's chains advanced by
 * fixed-trajectory HMC on the masked fold log density, with the online LogS
 * accumulators and the diagnostics computed from them.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU
 * baseline load this file's library (through oracle/c_oracle.py).  It shares
 * no code with the HIP library, nor with the numpy oracle beside it: both
 * oracles are written from the paper, and the tests hold them to each other
 * and to closed forms.
 *
 * What it computes, by the paper's passages:
 *  - fold roles (Appendix B masks; tri-state for hv-block): role_k(row) from
 *    a fold index, per-fold intervals or a dense K x n matrix;
 *  - the masked log density of chain c in fold k (Appendix B):
 *      log pi_c(theta) = log prior(theta) + sum_rows [train] l(y, eta),
 *    its gradient by the chain rule, and the log predictive density of the
 *    fold's test rows s_c(theta) = sum_rows [test] l(y, eta);
 *  - one HMC transition per chain (Section 3.3): momentum z / sqrt(M^-1)
 *    from Philox4x32-10 normals, S leapfrog steps of size eps, Metropolis
 *    test on the fp64 energy difference, divergence when it is not finite or
 *    the energy rose by more than 1000;
 *  - Algorithm A2's accumulators per chain: log-sum-exp of s (U) and of 2s
 *    (U2), batch sums Z folded into U, V, V2 at batch ends, and the shuffle
 *    blocks' statistics (Welford, or the shifted sums the algorithm writes);
 *  - the estimates of Sections 2.4 and 4 from those accumulators: elpd per
 *    fold (eqs est-e, cv-score), batch-means variance (eq bmvar), MCSE
 *    (eqs clt, mc-var), ESS and R-hat (eq rhat).
 * Every sum runs in ascending index order.
 *
 * Random numbers: Philox4x32-10 from its published definition (Salmon,
 * Moraes, Dror, Shaw, SC'11), key = (seed mod 2^32, seed div 2^32),
 * counter = (global chain id, iteration, purpose, block); purpose 1 =
 * momentum (block j gives coordinates 2j, 2j+1 by Box-Muller), purpose 2 =
 * accept (block 0).  A uniform from words (w0, w1) is
 * ((w0 2^32 + w1) >> 12) 2^-52 + 2^-53.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { FAM_GAUSS = 0, FAM_LOGIT = 1, FAM_POIS = 2, FAM_HLOGIT = 3, FAM_HGAUSS = 4 };
enum { ROLE_EXCL = 0, ROLE_TRAIN = 1, ROLE_TEST = 2 };
enum { FOLD_INDEX = 0, FOLD_INTERVALS = 1, FOLD_DENSE = 2 };

#define HALF_NORMAL_VAR 10.0     /* variance of the two scale priors of the hierarchical Gaussian */
#define DIVERGENCE 1000.0

typedef struct {
  int32_t family;
  int64_t n, p, d;
  int32_t K, L;
  const double* X;            /* n x p, row-major */
  const double* y;            /* n */
  int32_t fold_kind;
  const int32_t* fold_index;  /* n */
  const int64_t* intervals;   /* K x 4: test_lo, test_hi, excl_lo, excl_hi */
  const int8_t* roles;        /* K x n */
  int32_t n_groups;
  const int32_t* group_of;    /* n */
  double sigma;
  const double* prior_scale;  /* p */
  const double* inv_mass;     /* d */
  double step_size;
  int32_t n_leapfrog;
  uint64_t seed;
  int64_t chain_offset;
  int32_t n_warmup, batch_size, n_blocks, batches_per_block, rhat_mode;
} pco_model;

typedef struct {
  double *Z, *U, *U2, *V, *V2;   /* C each */
  int64_t* blk_n;                /* C x D */
  double *blk_mean, *blk_m2;     /* C x D */
  int64_t *n_accept, *n_divergent;
  double *wsum, *center;         /* C (shifted-sums mode) */
  int64_t n_wu, n_draws;
} pco_acc;

static const double PI = 3.14159265358979323846;
static const double LN2 = 0.69314718055994530942;
static const double LOG_2PI = 1.8378770664093453;   /* log(2 pi) */

/* ---- Philox4x32-10 --------------------------------------------------------- */
void pco_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t* out) {
  uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t a = (uint64_t)0xD2511F53u * x0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t n0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
    const uint32_t n2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)b;
    x3 = (uint32_t)a;
    x0 = n0;
    x2 = n2;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

static double uniform01(uint32_t w0, uint32_t w1) {
  const uint64_t bits = ((uint64_t)w0 << 32) | w1;
  return (double)(bits >> 12) * 0x1p-52 + 0x1p-53;
}

/* ---- fold roles ------------------------------------------------------------ */
static int role_of(const pco_model* m, int k, int64_t row) {
  if (m->fold_kind == FOLD_INDEX) return m->fold_index[row] == k ? ROLE_TEST : ROLE_TRAIN;
  if (m->fold_kind == FOLD_INTERVALS) {
    const int64_t* iv = m->intervals + 4 * (int64_t)k;
    if (row >= iv[0] && row < iv[1]) return ROLE_TEST;
    if (row >= iv[2] && row < iv[3]) return ROLE_EXCL;
    return ROLE_TRAIN;
  }
  return m->roles[(int64_t)k * m->n + row];
}

/* log(e^a + e^b), as the paper's streaming log-sum-exp needs it */
static double logaddexp(double a, double b) {
  if (a == b) return a + LN2;       /* also -inf + -inf */
  const double t = a - b;
  if (t > 0) return a + log1p(exp(-t));
  if (t <= 0) return b + log1p(exp(t));
  return t;                           /* NaN */
}

static double sigmoid(double e) {
  if (e >= 0) return 1.0 / (1.0 + exp(-e));
  const double z = exp(e);
  return z / (1.0 + z);
}

static int hierarchical(int fam) { return fam == FAM_HLOGIT || fam == FAM_HGAUSS; }

/* first coordinate of the group effects z */
static int64_t z_first(const pco_model* m) { return m->p + (m->family == FAM_HGAUSS ? 3 : 2); }

/* log half-normal density with variance v at x > 0 */
static double log_half_normal(double x, double v) { return LN2 - 0.5 * log(2.0 * PI * v) - x * x / (2.0 * v); }

/* log prior and (if g) its gradient, added to g */
static double log_prior(const pco_model* m, const double* th, double* g) {
  double lp = 0.0;
  if (m->family == FAM_HLOGIT || m->family == FAM_HGAUSS) {
    const int64_t p = m->p;
    for (int64_t j = 0; j < m->d; ++j) {
      const int scale = (j == p + 1) || (m->family == FAM_HGAUSS && j == p + 2);
      if (!scale) {
        lp += -0.5 * LOG_2PI - 0.5 * th[j] * th[j];
        if (g) g[j] += -th[j];
      } else {
        const double u = th[j], s = exp(u);
        const double v = m->family == FAM_HGAUSS ? HALF_NORMAL_VAR : 1.0;
        lp += log_half_normal(s, v) + u;          /* the log-Jacobian of s = e^u */
        if (g) g[j] += -s * s / v + 1.0;
      }
    }
    return lp;
  }
  for (int64_t j = 0; j < m->p; ++j) {
    const double s = m->prior_scale[j], t = th[j] / s;
    lp += -0.5 * LOG_2PI - log(s) - 0.5 * t * t;
    if (g) g[j] += -th[j] / (s * s);
  }
  return lp;
}

/* One chain in fold k at theta: log density, its gradient (if g; g has d
 * entries, overwritten) and the log predictive of the test rows (if s).
 * pg: n_groups scratch entries (hierarchical families). */
static void eval_chain(const pco_model* m, int k, const double* th, double* logp, double* g, double* s, double* pg) {
  const int64_t n = m->n, p = m->p;
  const int fam = m->family;
  const int hier = hierarchical(fam);
  const int64_t z0 = hier ? z_first(m) : 0;
  const double mu = hier ? th[p] : 0.0;
  const double tau = hier ? exp(th[p + 1]) : 0.0;
  const double sy = fam == FAM_HGAUSS ? exp(th[p + 2]) : m->sigma;
  const double ll_const = fam == FAM_HGAUSS ? -0.5 * LOG_2PI - th[p + 2] : -0.5 * log(2.0 * PI * m->sigma * m->sigma);
  double ll = 0.0, lpred = 0.0, gmu = 0.0, guy = 0.0;
  if (g) memset(g, 0, sizeof(double) * (size_t)m->d);
  if (g && hier) memset(pg, 0, sizeof(double) * (size_t)m->n_groups);
  for (int64_t row = 0; row < n; ++row) {
    const int role = role_of(m, k, row);
    if (role == ROLE_EXCL) continue;
    if (role == ROLE_TEST && !s) continue;
    const double* x = m->X + row * p;
    double eta = 0.0;
    for (int64_t j = 0; j < p; ++j) eta += x[j] * th[j];
    if (hier) eta += mu + tau * th[z0 + m->group_of[row]];
    const double yv = m->y[row];
    double l, r;
    if (fam == FAM_GAUSS || fam == FAM_HGAUSS) {
      const double e = yv - eta;
      l = ll_const - e * e / (2.0 * sy * sy);
      r = e / (sy * sy);
    } else if (fam == FAM_POIS) {
      const double lam = exp(eta);
      l = yv * eta - lam - lgamma(yv + 1.0);
      r = yv - lam;
    } else {
      l = yv * eta - logaddexp(0.0, eta);
      r = yv - sigmoid(eta);
    }
    if (role == ROLE_TEST) {
      lpred += l;
      continue;
    }
    ll += l;
    if (!g) continue;
    for (int64_t j = 0; j < p; ++j) g[j] += r * x[j];
    if (hier) {
      gmu += r;
      pg[m->group_of[row]] += r;
      if (fam == FAM_HGAUSS) {
        const double e = yv - eta;
        guy += e * e / (sy * sy) - 1.0;
      }
    }
  }
  if (g && hier) {
    double gu = 0.0;
    for (int gi = 0; gi < m->n_groups; ++gi) {
      g[z0 + gi] = tau * pg[gi];
      gu += pg[gi] * th[z0 + gi];
    }
    g[p] = gmu;
    g[p + 1] = tau * gu;
    if (fam == FAM_HGAUSS) g[p + 2] = guy;
  }
  if (logp) *logp = ll + log_prior(m, th, g);
  if (s) *s = lpred;
}

/* ---- batched evaluation (test hook) ---------------------------------------- */
int pco_log_density(const pco_model* m, int64_t C, const double* theta, double* logp, double* grad, double* s,
                    int threads) {
  int bad = 0;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
  {
    double* pg = (double*)malloc(sizeof(double) * (size_t)(m->n_groups > 0 ? m->n_groups : 1));
    if (!pg) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(static)
    for (int64_t c = 0; c < C; ++c) {
      if (!pg) continue;
      eval_chain(m, (int)(c / m->L), theta + c * m->d, logp ? logp + c : NULL, grad ? grad + c * m->d : NULL,
                 s ? s + c : NULL, pg);
    }
    free(pg);
  }
  return bad ? -1 : 0;
}

/* ---- one HMC transition of chain c at iteration t --------------------------- */
typedef struct {
  double *p, *q1, *g1, *pg;
} scratch;

static void transition(const pco_model* m, int64_t c, int64_t t, double* q, double* logp, double* g, double* s,
                       int* accepted, int* divergent, scratch* w) {
  const int64_t d = m->d;
  const int k = (int)(c / m->L);
  const uint32_t gid = (uint32_t)(m->chain_offset + c);
  const double eps = m->step_size;
  /* momentum p = z / sqrt(M^-1), kinetic energy 1/2 sum M^-1 p^2 */
  double k0 = 0.0;
  for (int64_t jb = 0; 2 * jb < d; ++jb) {
    uint32_t wv[4];
    pco_philox(m->seed, gid, (uint32_t)t, 1u, (uint32_t)jb, wv);
    const double u1 = uniform01(wv[0], wv[1]), u2 = uniform01(wv[2], wv[3]);
    const double rr = sqrt(-2.0 * log(u1));
    const double z[2] = {rr * cos(2.0 * PI * u2), rr * sin(2.0 * PI * u2)};
    for (int h = 0; h < 2 && 2 * jb + h < d; ++h) {
      const int64_t j = 2 * jb + h;
      w->p[j] = z[h] / sqrt(m->inv_mass[j]);
    }
  }
  for (int64_t j = 0; j < d; ++j) k0 += m->inv_mass[j] * w->p[j] * w->p[j];
  const double h0 = -*logp + 0.5 * k0;
  /* leapfrog from (q, p) with the carried gradient */
  memcpy(w->q1, q, sizeof(double) * (size_t)d);
  memcpy(w->g1, g, sizeof(double) * (size_t)d);
  for (int64_t j = 0; j < d; ++j) w->p[j] += 0.5 * eps * w->g1[j];
  double lp1 = 0.0;
  for (int step = 0; step < m->n_leapfrog; ++step) {
    for (int64_t j = 0; j < d; ++j) w->q1[j] += eps * m->inv_mass[j] * w->p[j];
    eval_chain(m, k, w->q1, &lp1, w->g1, NULL, w->pg);
    const double h = step < m->n_leapfrog - 1 ? eps : 0.5 * eps;
    for (int64_t j = 0; j < d; ++j) w->p[j] += h * w->g1[j];
  }
  double k1 = 0.0;
  for (int64_t j = 0; j < d; ++j) k1 += m->inv_mass[j] * w->p[j] * w->p[j];
  const double log_ratio = h0 - (-lp1 + 0.5 * k1);
  uint32_t wa[4];
  pco_philox(m->seed, gid, (uint32_t)t, 2u, 0u, wa);
  const double u = uniform01(wa[0], wa[1]);
  const int finite = isfinite(log_ratio);
  *accepted = finite && log(u) < log_ratio;
  *divergent = !finite || -log_ratio > DIVERGENCE;
  if (*accepted) {
    memcpy(q, w->q1, sizeof(double) * (size_t)d);
    memcpy(g, w->g1, sizeof(double) * (size_t)d);
    *logp = lp1;
    eval_chain(m, k, q, NULL, NULL, s, w->pg);
  }
}

/* ---- Algorithm A2's accumulators -------------------------------------------- */
static void accumulate(const pco_model* m, pco_acc* a, int64_t c, double s, int64_t i) {
  const int D = m->n_blocks, b = m->batch_size;
  a->Z[c] = logaddexp(a->Z[c], s);
  a->U2[c] = logaddexp(a->U2[c], 2.0 * s);
  int64_t blk = i / ((int64_t)m->batches_per_block * b);
  if (blk > D - 1) blk = D - 1;
  const int64_t e = c * D + blk;
  a->blk_n[e] += 1;
  if (m->rhat_mode == 1) {
    const double dv = s - a->center[c];
    a->blk_mean[e] += dv;
    a->blk_m2[e] += dv * dv;
  } else {
    const double delta = s - a->blk_mean[e];
    a->blk_mean[e] += delta / (double)a->blk_n[e];
    a->blk_m2[e] += delta * (s - a->blk_mean[e]);
  }
  if ((i + 1) % b == 0) {
    a->U[c] = logaddexp(a->U[c], a->Z[c]);
    a->V[c] = logaddexp(a->V[c], a->Z[c] - log((double)b));
    a->V2[c] = logaddexp(a->V2[c], 2.0 * a->Z[c] - 2.0 * log((double)b));
    a->Z[c] = -INFINITY;
  }
}

/* shifted-sums mode: C_k = mean of the fold's warm-up draws (0 without warm-up) */
static void fix_center(const pco_model* m, pco_acc* a) {
  for (int k = 0; k < m->K; ++k) {
    double sum = 0.0;
    for (int l = 0; l < m->L; ++l) sum += a->wsum[(int64_t)k * m->L + l];
    const double ck = a->n_wu > 0 ? sum / ((double)m->L * (double)a->n_wu) : 0.0;
    for (int l = 0; l < m->L; ++l) a->center[(int64_t)k * m->L + l] = ck;
  }
}

/* Initial state at init_pos [C x d] and empty accumulators. */
int pco_start(const pco_model* m, const double* init_pos, double* q, double* logp, double* grad, double* s,
              pco_acc* a, int threads) {
  const int64_t C = (int64_t)m->K * m->L;
  memcpy(q, init_pos, sizeof(double) * (size_t)(C * m->d));
  if (pco_log_density(m, C, q, logp, grad, s, threads) != 0) return -1;
  for (int64_t c = 0; c < C; ++c) {
    a->Z[c] = a->U[c] = a->U2[c] = a->V[c] = a->V2[c] = -INFINITY;
    a->n_accept[c] = a->n_divergent[c] = 0;
    a->wsum[c] = a->center[c] = 0.0;
  }
  memset(a->blk_n, 0, sizeof(int64_t) * (size_t)(C * m->n_blocks));
  memset(a->blk_mean, 0, sizeof(double) * (size_t)(C * m->n_blocks));
  memset(a->blk_m2, 0, sizeof(double) * (size_t)(C * m->n_blocks));
  a->n_wu = 0;
  a->n_draws = 0;
  if (m->n_warmup == 0) fix_center(m, a);
  return 0;
}

/* Advance every chain from global iteration t0 by n_iter transitions. */
int pco_advance(const pco_model* m, int64_t t0, int64_t n_iter, double* q, double* logp, double* grad, double* s,
                pco_acc* a, int threads) {
  const int64_t C = (int64_t)m->K * m->L, d = m->d;
  int* acc = (int*)malloc(sizeof(int) * (size_t)C);
  int* div = (int*)malloc(sizeof(int) * (size_t)C);
  if (!acc || !div) {
    free(acc);
    free(div);
    return -1;
  }
  int bad = 0;
  for (int64_t t = t0; t < t0 + n_iter && !bad; ++t) {
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
      scratch w;
      w.p = (double*)malloc(sizeof(double) * (size_t)d);
      w.q1 = (double*)malloc(sizeof(double) * (size_t)d);
      w.g1 = (double*)malloc(sizeof(double) * (size_t)d);
      w.pg = (double*)malloc(sizeof(double) * (size_t)(m->n_groups > 0 ? m->n_groups : 1));
      const int ok = w.p && w.q1 && w.g1 && w.pg;
      if (!ok) {
#pragma omp atomic write
        bad = 1;
      }
#pragma omp for schedule(static)
      for (int64_t c = 0; c < C; ++c) {
        if (!ok) continue;
        transition(m, c, t, q + c * d, logp + c, grad + c * d, s + c, acc + c, div + c, &w);
      }
      free(w.p);
      free(w.q1);
      free(w.g1);
      free(w.pg);
    }
    if (bad) break;
    if (t < m->n_warmup) {
      if (m->rhat_mode == 1) {
        for (int64_t c = 0; c < C; ++c) a->wsum[c] += s[c];
        a->n_wu += 1;
      }
      if (t + 1 == m->n_warmup) fix_center(m, a);
    } else {
      const int64_t i = t - m->n_warmup;
      for (int64_t c = 0; c < C; ++c) {
        accumulate(m, a, c, s[c], i);
        a->n_accept[c] += acc[c];
        a->n_divergent[c] += div[c];
      }
      a->n_draws = i + 1;
    }
  }
  free(acc);
  free(div);
  return bad ? -1 : 0;
}

/* ---- estimates and diagnostics from the accumulators ------------------------ */

/* per chain (n, mean, M2) of s over the blocks: Chan's merge of the Welford
 * blocks, or the shifted sums (mean relative to C_k, which R-hat does not see) */
static void chain_moments(const pco_model* m, const pco_acc* a, int64_t c, double* n, double* mean, double* m2) {
  const int D = m->n_blocks;
  double nn = 0.0, mu = 0.0, M2 = 0.0;
  if (m->rhat_mode == 1) {
    double y = 0.0, y2 = 0.0;
    for (int b = 0; b < D; ++b) {
      nn += (double)a->blk_n[c * D + b];
      y += a->blk_mean[c * D + b];
      y2 += a->blk_m2[c * D + b];
    }
    mu = nn > 0 ? y / nn : 0.0;
    M2 = y2 - (nn > 0 ? y * y / nn : 0.0);
  } else {
    for (int b = 0; b < D; ++b) {
      const double nb = (double)a->blk_n[c * D + b];
      const double tot = nn + nb;
      if (tot > 0) {
        const double delta = a->blk_mean[c * D + b] - mu;
        mu = mu + delta * (nb / tot);
        M2 = M2 + a->blk_m2[c * D + b] + delta * delta * nn * nb / tot;
      }
      nn = tot;
    }
  }
  *n = nn;
  *mean = mu;
  *m2 = M2;
}

/* over one fold's L values x and x2: max m of x, s1 = sum e^{x-m},
 * bracket = sum e^{x2-2m} - s1^2 / n_terms */
static void fold_terms(const double* x, const double* x2, int L, double n_terms, double* mx, double* s1,
                       double* bracket) {
  double m = -INFINITY;
  for (int l = 0; l < L; ++l)
    if (x[l] > m) m = x[l];
  double a = 0.0, b = 0.0;
  for (int l = 0; l < L; ++l) {
    a += exp(x[l] - m);
    b += exp(x2[l] - 2.0 * m);
  }
  *mx = m;
  *s1 = a;
  *bracket = b - a * a / n_terms;
}

/* out[6]: elpd, mcse, rhat_max, ess, accept_rate, n_divergent.  Per fold
 * arrays (K entries) may be NULL. */
int pco_diagnostics(const pco_model* m, const pco_acc* a, double* elpd_fold, double* mcse_fold, double* rhat_fold,
                    double* ess_fold, double* out) {
  const int K = m->K, L = m->L, b = m->batch_size;
  const int64_t N = a->n_draws, C = (int64_t)K * L;
  const double LN = (double)L * (double)N;
  const int64_t nbatch = N / b;
  double* Uall = (double*)malloc(sizeof(double) * (size_t)L);
  double* mean_l = (double*)malloc(sizeof(double) * (size_t)L);
  if (!Uall || !mean_l) {
    free(Uall);
    free(mean_l);
    return -1;
  }
  double elpd = 0.0, var_sum = 0.0, rmax = -INFINITY, s2sum = 0.0, sig2sum = 0.0;
  for (int k = 0; k < K; ++k) {
    const int64_t c0 = (int64_t)k * L;
    for (int l = 0; l < L; ++l) Uall[l] = logaddexp(a->U[c0 + l], a->Z[c0 + l]);
    /* elpd_k = log sum_l e^{U_l} - log(LN) */
    double mU, t1, brU;
    fold_terms(Uall, a->U2 + c0, L, LN, &mU, &t1, &brU);
    const double ek = N > 0 ? mU + log(t1) - log(LN) : NAN;
    /* R-hat from the chains' moments */
    double rk = NAN;
    if (N >= 2) {
      double W = 0.0, grand = 0.0, B = 0.0;
      for (int l = 0; l < L; ++l) {
        double nn, mu, M2;
        chain_moments(m, a, c0 + l, &nn, &mu, &M2);
        mean_l[l] = mu;
        W += M2 / ((double)N - 1.0);
        grand += mu;
      }
      W /= L;
      grand /= L;
      for (int l = 0; l < L; ++l) B += (mean_l[l] - grand) * (mean_l[l] - grand);
      B *= (double)N / (L - 1.0);
      rk = sqrt(((double)N - 1.0) / (double)N + B / ((double)N * W));
    }
    /* pooled variance of f = e^s and batch-means variance, both relative to fhat^2 */
    const double log_fhat = mU + log(t1) - log(LN);
    const double s2_rel = exp(2.0 * mU + log(brU > 0 ? brU : 0.0) - log(LN - 1.0) - 2.0 * log_fhat);
    double sig2_rel = NAN;
    if (nbatch >= 1 && (double)L * nbatch > 1) {
      double mV, v1, brV;
      fold_terms(a->V + c0, a->V2 + c0, L, (double)L * nbatch, &mV, &v1, &brV);
      sig2_rel = exp(log((double)b) - log((double)L * nbatch - 1.0) + 2.0 * mV + log(brV > 0 ? brV : 0.0) -
                     2.0 * log_fhat);
    }
    const double var_rel = sig2_rel / LN;
    if (elpd_fold) elpd_fold[k] = ek;
    if (mcse_fold) mcse_fold[k] = sqrt(var_rel);
    if (rhat_fold) rhat_fold[k] = rk;
    if (ess_fold) ess_fold[k] = LN * s2_rel / sig2_rel;
    elpd += ek;
    var_sum += var_rel;
    if (isnan(rk)) rmax = NAN;
    else if (!isnan(rmax) && rk > rmax) rmax = rk;
    s2sum += s2_rel;
    sig2sum += sig2_rel;
  }
  free(Uall);
  free(mean_l);
  int64_t na = 0, nd = 0;
  for (int64_t c = 0; c < C; ++c) {
    na += a->n_accept[c];
    nd += a->n_divergent[c];
  }
  out[0] = elpd;
  out[1] = sqrt(var_sum);
  out[2] = rmax;
  out[3] = LN * s2sum / sig2sum;
  out[4] = (double)na / (double)(C * N > 0 ? C * N : 1);
  out[5] = (double)nd;
  return 0;
}
