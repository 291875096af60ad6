// Fused VALU path: one workgroup owns 64 chains (one per lane) and runs whole
// HMC transitions for them -- momentum, S masked value/gradient evaluations
// with the leapfrog updates, Metropolis test, log predictive and
// accumulation -- without any grid-wide synchronisation, because chains never
// interact (Section 3.3).  The W waves of the workgroup split the rows; each
// row of X is read once per wave with scalar loads and broadcast to the 64
// chains.  Used for narrow designs (p <= 64).
#include <type_traits>

#include "pcv_internal.h"

namespace pcv {

enum { MODE_ITER = 0, MODE_GRAD = 1, MODE_LEAP = 2, MODE_PART = 3 };

struct ValuArgs {
  DevModel m;
  const void* Xv;    // [n][PB] padded copy of X in T
  int64_t t0;
  int n_iter;
  int mode;
  int n_steps;
  // MODE_PART (row splits): partial sums [split][R][C], R = p (+ groups), and
  // partial values [split][C]
  double* Gpart;
  double* Vpart;
  int value;
  double* uscr;   // hierarchical: [C] log tau at the evaluation point (split 0 writes it)
  int series;     // MODE_PART, GLM families: X holds the lags of y (see grad_eval)
};

template <typename T>
struct ValuY;
template <>
struct ValuY<double> {
  static __device__ __forceinline__ double get(const DevModel& m, int64_t i) { return m.y64[i]; }
};
template <>
struct ValuY<float> {
  static __device__ __forceinline__ float get(const DevModel& m, int64_t i) { return m.y32[i]; }
};

template <int FAM, typename T>
__device__ __forceinline__ T vresid(T y, T eta, T is2) {
  if constexpr (sizeof(T) == 8) return resid64<FAM>(y, eta, is2);
  else return resid32<FAM>(y, eta, is2);
}
template <int FAM, typename T>
__device__ __forceinline__ T vell0(T y, T eta, T is2) {
  if constexpr (sizeof(T) == 8) return ell0_64<FAM>(y, eta, is2);
  else return ell0_32<FAM>(y, eta, is2);
}

// Workgroup-wide gradient (and optionally value) of log pi at q1 for the 64
// chains of this workgroup.  On return wave 0 holds the likelihood gradient in
// G (beta part) and, for the hierarchical family, the per-group residual sums
// in LDS rg; val (wave 0) holds the masked log-likelihood sum without row
// constants.
// Coefficients per round of the cross-wave gradient reduction (LDS [W][JC][64]).
template <typename T, int PB>
__host__ __device__ constexpr int valu_jc() {
  return (sizeof(T) == 8 ? 4 : 8) < PB ? (sizeof(T) == 8 ? 4 : 8) : PB;
}

// Row-loop fold test for rows on which every lane of the wave trains.
constexpr int ALL_TRAIN = -1;

// Groups [glo, ghi] spanned by the rows [wr[0], wr[W]) of a workgroup (rows
// are sorted by group); empty range (glo > ghi) when it has no rows.
__device__ __forceinline__ void block_groups(const DevModel& m, const int32_t* wr, int W, int& glo, int& ghi) {
  glo = 0;
  ghi = -1;
  if (wr[W] > wr[0]) {
    glo = m.group_of[wr[0]];
    ghi = m.group_of[wr[W] - 1];
  }
}

// FAM_HGAUSS also returns (wave 0) qsum = sum over training rows of
// (y - eta)^2 / sigma_y^2, from which the log sigma_y gradient follows.
template <typename T, int FAM, int PB, bool VALUE>
__device__ __forceinline__ void grad_eval(const DevModel& m, const T* __restrict__ Xv, int lane, int wave,
                                          int W, int64_t cc, int k, int elo, int ehi, T (&G)[PB],
                                          double& val, double& qsum, char* smem, bool want_value = true,
                                          const int32_t* wave_rows = nullptr, bool series = false) {
  constexpr int JC = valu_jc<T, PB>();
  T* red = reinterpret_cast<T*>(smem);                                      // [W][JC][64]
  double* vred = reinterpret_cast<double*>(smem + sizeof(T) * W * JC * 64);  // [W][64]
  T* zt = reinterpret_cast<T*>(smem + sizeof(T) * W * JC * 64 + sizeof(double) * W * 64);  // [G][64]
  T* rg = zt + (hier_fam<FAM>() ? m.n_groups * 64 : 0);                      // [G][64]
  T* gfin = rg + (hier_fam<FAM>() ? m.n_groups * 64 : 0);                    // [PB][64]
  T* ef = gfin + PB * 64;                                                     // [W][2][64]
  int* eg = reinterpret_cast<int*>(ef + (hier_fam<FAM>() ? W * 2 * 64 : 0));  // [W][2]

  const int32_t* wr = wave_rows ? wave_rows : m.wave_rows;
  T th[PB];
  theta_row<PB>(m, m.q1, cc, th);
  T mu = 0;
  if (hier_fam<FAM>()) {
    // tau z_g only for the groups of this workgroup's rows; rg cleared for all
    mu = static_cast<T>(m.q1[m.p * m.C + cc]);
    const T tau = static_cast<T>(exp(m.q1[(m.p + 1) * m.C + cc]));
    const int64_t z0 = hier_z0(m);
    int glo, ghi;
    block_groups(m, wr, W, glo, ghi);
    for (int g = glo + wave; g <= ghi; g += W)
      zt[g * 64 + lane] = tau * static_cast<T>(m.q1[(z0 + g) * m.C + cc]);
    for (int g = wave; g < m.n_groups; g += W) rg[g * 64 + lane] = T(0);
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < PB; ++j) G[j] = T(0);
  val = 0.0;
  qsum = 0.0;
  // the chain's own 1/sigma_y^2 for the hierarchical Gaussian
  const T is2 = FAM == FAM_HGAUSS ? static_cast<T>(exp(-2.0 * m.q1[(m.p + 2) * m.C + cc]))
                                  : static_cast<T>(m.inv_sigma2);
  T qacc = T(0);
  const int64_t r0 = wr[wave], r1 = wr[wave + 1];
  // Hierarchical: rows are sorted by group.  A group that starts and ends
  // inside this wave's rows is this wave's alone and goes straight to rg; the
  // wave's first and last groups may be shared with its neighbours and go to
  // edge slots, added to rg in a fixed order after the loop.
  int gcur = -1, gfirst = -1;
  T racc = T(0), zcur = T(0);
  // One row: its coefficients xv, response y, group g and fold id f (the
  // fold id is used by index-coded folds only); the fold encoding is a
  // compile-time constant of the row loop that calls it.
  auto row = [&](auto fold_kind, int64_t i, const T (&xv)[PB], T y, int g, int f) {
    constexpr int FKR = decltype(fold_kind)::value;
    T eta = T(0);
#pragma unroll
    for (int j = 0; j < PB; ++j) eta += xv[j] * th[j];
    if (hier_fam<FAM>()) {
      if (g != gcur) {
        if (gcur >= 0) {
          if (gfirst < 0) {
            gfirst = gcur;
            ef[(wave * 2) * 64 + lane] = racc;
          } else {
            rg[gcur * 64 + lane] += racc;
          }
        }
        gcur = g;
        racc = T(0);
        zcur = zt[g * 64 + lane];
      }
      eta += mu + zcur;
    }
    bool train;
    if constexpr (FKR == ALL_TRAIN) train = true;
    else if constexpr (FKR == PCV_FOLDS_INDEX) train = f != k;
    else if constexpr (FKR == PCV_FOLDS_INTERVALS) train = (i < elo) || (i >= ehi);
    else train = m.roles[static_cast<int64_t>(k) * m.n + i] == 1;
    const T r = train ? vresid<FAM, T>(y, eta, is2) : T(0);
#pragma unroll
    for (int j = 0; j < PB; ++j) G[j] += xv[j] * r;
    if (hier_fam<FAM>()) racc += r;
    if (FAM == FAM_HGAUSS) qacc += (y - eta) * r;
    if (VALUE && want_value) {
      if (train) val += static_cast<double>(vell0<FAM, T>(y, eta, is2));
    }
  };
  // the fold encoding is decided once, outside the row loop
  auto rows = [&](auto fold_kind, int64_t ra, int64_t rb) {
    constexpr int FKR = decltype(fold_kind)::value;
    // GLM rows: four rows per trip puts their scalar loads under one wait.
    // The hierarchical row carries a group-change branch and gains nothing.
    constexpr int RU = hier_fam<FAM>() ? 1 : 4;
    if constexpr (!hier_fam<FAM>()) {
      // Autoregressive design (p = PB lags of the response): row i + 1's
      // coefficients are row i's response followed by row i's first PB - 1
      // coefficients, so after the first row of the range only responses
      // are loaded and the coefficients slide through registers.  The host
      // checks the identity exactly; the values and their order are those
      // of the general loop below.
      if (series) {
        if (ra >= rb) return;
        T xv[PB];
#pragma unroll
        for (int j = 0; j < PB; ++j) xv[j] = Xv[ra * PB + j];
#pragma unroll RU
        for (int64_t i = ra; i < rb; ++i) {
          const T y = ValuY<T>::get(m, i);
          row(fold_kind, i, xv, y, 0, FKR == PCV_FOLDS_INDEX ? m.fold_index[i] : 0);
#pragma unroll
          for (int j = PB - 1; j > 0; --j) xv[j] = xv[j - 1];
          xv[0] = y;
        }
        return;
      }
    }
#pragma unroll RU
    for (int64_t i = ra; i < rb; ++i) {
      const T* xr = Xv + i * PB;
      T xv[PB];
#pragma unroll
      for (int j = 0; j < PB; ++j) xv[j] = xr[j];
      row(fold_kind, i, xv, ValuY<T>::get(m, i), hier_fam<FAM>() ? m.group_of[i] : 0,
          FKR == PCV_FOLDS_INDEX ? m.fold_index[i] : 0);
    }
  };
  if (m.fold_kind == PCV_FOLDS_INDEX) {
    rows(std::integral_constant<int, PCV_FOLDS_INDEX>{}, r0, r1);
  } else if (m.fold_kind == PCV_FOLDS_INTERVALS && hier_fam<FAM>()) {
    rows(std::integral_constant<int, PCV_FOLDS_INTERVALS>{}, r0, r1);
  } else if (m.fold_kind == PCV_FOLDS_INTERVALS) {
    // Interval folds exclude one contiguous row range per lane.  Outside the
    // union hull [xlo, xhi) of the wave's ranges every lane trains on every
    // row, so those rows skip the per-lane test; same rows, same order.
    // (GLM families only: the extra row loops cost the hierarchical kernel
    // registers.)
    int xlo = elo < ehi ? elo : INT32_MAX, xhi = elo < ehi ? ehi : INT32_MIN;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      xlo = min(xlo, __shfl_xor(xlo, o));
      xhi = max(xhi, __shfl_xor(xhi, o));
    }
    xlo = __builtin_amdgcn_readfirstlane(xlo);
    xhi = __builtin_amdgcn_readfirstlane(xhi);
    const int64_t ra = xlo < r0 ? r0 : (xlo > r1 ? r1 : static_cast<int64_t>(xlo));
    const int64_t rb = xhi < ra ? ra : (xhi > r1 ? r1 : static_cast<int64_t>(xhi));
    rows(std::integral_constant<int, ALL_TRAIN>{}, r0, ra);
    rows(std::integral_constant<int, PCV_FOLDS_INTERVALS>{}, ra, rb);
    rows(std::integral_constant<int, ALL_TRAIN>{}, rb, r1);
  } else {
    rows(std::integral_constant<int, PCV_FOLDS_DENSE>{}, r0, r1);
  }
  if (hier_fam<FAM>()) {
    int glast = -1;
    if (gcur >= 0) {
      if (gfirst < 0) {
        gfirst = gcur;
        ef[(wave * 2) * 64 + lane] = racc;
      } else {
        glast = gcur;
        ef[(wave * 2 + 1) * 64 + lane] = racc;
      }
    }
    if (lane == 0) {
      eg[2 * wave] = gfirst;
      eg[2 * wave + 1] = glast;
    }
    __syncthreads();
    if (wave == 0) {
      for (int w = 0; w < W; ++w) {
        const int g0 = eg[2 * w], g1 = eg[2 * w + 1];
        if (g0 >= 0) rg[g0 * 64 + lane] += ef[(2 * w) * 64 + lane];
        if (g1 >= 0) rg[g1 * 64 + lane] += ef[(2 * w + 1) * 64 + lane];
      }
    }
    __syncthreads();
  }

  // Cross-wave reduction in a fixed order (bit-reproducible).
#pragma unroll
  for (int j0 = 0; j0 < PB; j0 += JC) {
    if (j0 < m.p) {
#pragma unroll
      for (int jj = 0; jj < JC; ++jj) red[(wave * JC + jj) * 64 + lane] = G[j0 + jj];
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
          T s = T(0);
          for (int w = 0; w < W; ++w) s += red[(w * JC + jj) * 64 + lane];
          gfin[(j0 + jj) * 64 + lane] = s;
        }
      }
      __syncthreads();
    }
  }
  if (VALUE && want_value) {
    vred[wave * 64 + lane] = val;
    __syncthreads();
    if (wave == 0) {
      double s = 0.0;
      for (int w = 0; w < W; ++w) s += vred[w * 64 + lane];
      val = s;
    }
    __syncthreads();
  }
  if (FAM == FAM_HGAUSS) {
    vred[wave * 64 + lane] = static_cast<double>(qacc);
    __syncthreads();
    if (wave == 0) {
      double s = 0.0;
      for (int w = 0; w < W; ++w) s += vred[w * 64 + lane];
      qsum = s;
    }
    __syncthreads();
  }
}

// Wave 0, lane = chain: add the prior to the reduced likelihood gradient
// (LDS gfin) and hand the full gradient to `emit(j, g)`.  The coordinate loop
// is deliberately not unrolled: unrolling hoists one address per coordinate
// out of the leapfrog loop and exhausts the register file.
template <typename T, int FAM, int PB, typename Emit>
__device__ __forceinline__ void finish_chain(const DevModel& m, int64_t c, int lane, char* smem, int W, double qsum,
                                             Emit emit) {
  constexpr int JC = valu_jc<T, PB>();
  T* zt = reinterpret_cast<T*>(smem + sizeof(T) * W * JC * 64 + sizeof(double) * W * 64);
  T* rg = zt + (hier_fam<FAM>() ? m.n_groups * 64 : 0);
  const T* gfin = rg + (hier_fam<FAM>() ? m.n_groups * 64 : 0);
  const uint8_t* mrow = mask_row(m, c);
#pragma nounroll
  for (int64_t j = 0; j < m.p; ++j)
    emit(j, (covariate_used(mrow, j) ? static_cast<double>(gfin[j * 64 + lane]) : 0.0) +
                prior_grad(m, m.q1[j * m.C + c], j));
  if (hier_fam<FAM>()) {
    const double u = m.q1[(m.p + 1) * m.C + c];
    const double tau = exp(u);
    const int64_t z0 = hier_z0(m);
    double gmu = 0.0, gu = 0.0;
#pragma nounroll
    for (int g = 0; g < m.n_groups; ++g) {
      const double rs = static_cast<double>(rg[g * 64 + lane]);
      const double z = m.q1[(z0 + g) * m.C + c];
      gmu += rs;
      gu += z * rs;
      emit(z0 + g, tau * rs - z);
    }
    emit(m.p, gmu - m.q1[m.p * m.C + c]);
    emit(m.p + 1, tau * gu + prior_grad(m, u, m.p + 1));
    if (FAM == FAM_HGAUSS) {
      // d/d log sigma_y of sum_train (-log sigma_y - (y - eta)^2 / (2 sigma_y^2))
      const double uy = m.q1[(m.p + 2) * m.C + c];
      emit(m.p + 2, qsum - m.ntrain[fold_of_chain(m, c)] + prior_grad(m, uy, m.p + 2));
    }
  }
}

// Per-workgroup setup shared by the three kernels below.
#define VALU_PROLOGUE                                                          \
  extern __shared__ __align__(16) char smem[];                                 \
  const DevModel& m = a.m;                                                     \
  const T* __restrict__ Xv = static_cast<const T*>(a.Xv);                      \
  const int lane = threadIdx.x & 63;                                           \
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);           \
  const int W = blockDim.x >> 6;                                               \
  const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + lane;              \
  const bool valid = c < m.C;                                                  \
  const int64_t cc = valid ? c : m.C - 1;                                      \
  const int k = fold_of_chain(m, cc);                                          \
  int elo = 0, ehi = 0;                                                        \
  if (m.fold_kind == PCV_FOLDS_INTERVALS) {                                    \
    elo = m.ivals[4 * k + 2];                                                  \
    ehi = m.ivals[4 * k + 3];                                                  \
  }                                                                            \
  T G[PB];                                                                     \
  double val, qsum;                                                            \
  const bool lead = (wave == 0) && valid;

constexpr int VALU_MAX_THREADS = 512;

// Value and gradient at q1 -> g1, logp1.
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_grad(ValuArgs a) {
  VALU_PROLOGUE
  grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, qsum, smem);
  if (lead) {
    finish_chain<T, FAM, PB>(m, c, lane, smem, W, qsum, [&](int64_t j, double g) { m.g1[j * m.C + c] = g; });
    m.logp1[c] = val + m.fold_const[k] + prior_quad(m, m.q1, c);
  }
}

// n_steps leapfrog steps from (q1, pm): gradient at the start, first half
// kick and drift, then the steps (used to check single trajectories).
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_leap(ValuArgs a) {
  VALU_PROLOGUE
  grad_eval<T, FAM, PB, false>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, qsum, smem);
  if (lead) {
    finish_chain<T, FAM, PB>(m, c, lane, smem, W, qsum, [&](int64_t j, double g) {
      const int64_t o = j * m.C + c;
      const double p = m.pm[o] + 0.5 * m.eps * g;
      m.pm[o] = p;
      m.q1[o] += m.eps * m.minv[j] * p;
    });
  }
  __syncthreads();
  for (int s = 0; s < a.n_steps; ++s) {
    const bool last = s == a.n_steps - 1;
    grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, qsum, smem);
    if (lead) {
      finish_chain<T, FAM, PB>(m, c, lane, smem, W, qsum,
                               [&](int64_t j, double g) { leapfrog_update(m, c, j, g, last); });
      if (last) m.logp1[c] = val + m.fold_const[k] + prior_quad(m, m.q1, c);
    }
    __syncthreads();
  }
}

// n_iter whole HMC transitions starting at global iteration t0.
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_iter(ValuArgs a) {
  VALU_PROLOGUE
  for (int it = 0; it < a.n_iter; ++it) {
    const int64_t t = a.t0 + it;
    if (lead) momentum_and_first_drift(m, c, t);
    __syncthreads();
    for (int s = 0; s < m.S; ++s) {
      const bool last = s == m.S - 1;
      grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, qsum, smem, last);
      if (lead) {
        finish_chain<T, FAM, PB>(m, c, lane, smem, W, qsum,
                                 [&](int64_t j, double g) { leapfrog_update(m, c, j, g, last); });
        if (last) m.logp1[c] = val + m.fold_const[k] + prior_quad(m, m.q1, c);
      }
      __syncthreads();
    }
    if (lead) accept_and_accumulate<FAM>(m, c, t);
    __syncthreads();
  }
}

// Row-split gradient (few chains, many rows): workgroup (chain block x, split
// y) evaluates its split's rows for its 64 chains; its W waves divide the
// split.  Wave 0 writes the raw partial sums [split][d][C] -- sum x r per
// coefficient and, hierarchical, the group sums and their mu and log tau
// shares -- and the partial value; the splits are added in a fixed order
// by k_reduce (GLMs) or k_valu_finish (hierarchical).
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_part(ValuArgs a) {
  VALU_PROLOGUE
  const int sp = blockIdx.y;
  const int32_t* wr = m.wave_rows + static_cast<int64_t>(sp) * (W + 1);
  const bool series = a.series != 0;
  if (a.value) grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, qsum, smem, true, wr, series);
  else grad_eval<T, FAM, PB, false>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, qsum, smem, false, wr, series);
  if (lead) {
    constexpr int JC = valu_jc<T, PB>();
    T* zt = reinterpret_cast<T*>(smem + sizeof(T) * W * JC * 64 + sizeof(double) * W * 64);
    const T* rg = zt + (hier_fam<FAM>() ? m.n_groups * 64 : 0);
    const T* gfin = rg + (hier_fam<FAM>() ? m.n_groups * 64 : 0);
    double* out = a.Gpart + static_cast<int64_t>(sp) * m.d * m.C + c;
#pragma nounroll
    for (int64_t j = 0; j < m.p; ++j) out[j * m.C] = static_cast<double>(gfin[j * 64 + lane]);
    if (hier_fam<FAM>()) {
      const int64_t z0 = hier_z0(m);
      // group sums r_g of this split's groups only (the finish kernel reads
      // group g from the splits that span it), and the split's shares of the
      // mu and log tau likelihood gradients, sum_g r_g and sum_g z_g r_g
      int glo, ghi;
      block_groups(m, wr, W, glo, ghi);
      double sr = 0.0, szr = 0.0;
#pragma nounroll
      for (int g = glo; g <= ghi; ++g) {
        const double r = static_cast<double>(rg[g * 64 + lane]);
        out[(z0 + g) * m.C] = r;
        sr += r;
        szr += m.q1[(z0 + g) * m.C + c] * r;
      }
      out[m.p * m.C] = sr;
      out[(m.p + 1) * m.C] = szr;
      if (FAM == FAM_HGAUSS) out[(m.p + 2) * m.C] = qsum;   // this split's sum of (y - eta)^2 / sigma_y^2
      if (sp == 0) a.uscr[c] = m.q1[(m.p + 1) * m.C + c];
    }
    if (a.value) a.Vpart[static_cast<int64_t>(sp) * m.C + c] = val;
  }
}

#if !defined(PCV_VALU_T)
// Hierarchical family, row splits: one thread per (entry, chain) of the
// [split][d][C] partials.  Coefficients, mu and log tau add every split,
// group g the splits that span it (gsplit), in split order; then the prior
// and the chain rule (mu: sum r - mu; log tau: tau sum z r + prior; z_g:
// tau r_g - z_g) with tau from uscr, the log tau the partials were taken
// at (q1 itself may already be updated by the log tau thread).  mode 0
// writes g1, 1 and 2 apply a (last) leapfrog update.
__global__ void k_valu_finish(DevModel m, const double* __restrict__ Gpart, const double* __restrict__ uscr, int ns,
                              int mode) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= m.d * m.C) return;
  const int64_t j = idx / m.C, c = idx - j * m.C;
  const int64_t dC = m.d * m.C;
  int s0 = 0, s1 = ns - 1;
  const int64_t z0 = hier_z0(m);
  if (j >= z0) {
    const int64_t g = j - z0;
    s0 = m.gsplit[2 * g];
    s1 = m.gsplit[2 * g + 1];
  }
  const double* gp = Gpart + idx;
  double v = 0.0;
  int sp = s0;
  for (; sp + 16 <= s1 + 1; sp += 16) {   // loads issued sixteen at a time, added in split order
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = gp[(sp + u) * dC];
#pragma unroll
    for (int u = 0; u < 16; ++u) v += t[u];
  }
  if (sp + 8 <= s1 + 1) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = gp[(sp + u) * dC];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
    sp += 8;
  }
  for (; sp <= s1; ++sp) v += gp[sp * dC];
  double g;
  if (j < m.p) {
    if (!covariate_used(mask_row(m, c), j)) v = 0.0;   // a masked coefficient: prior only
    g = v + prior_grad(m, m.q1[idx], j);
  } else if (j == m.p) {
    g = v - m.q1[idx];
  } else if (m.family == FAM_HGAUSS && j == m.p + 2) {
    // log sigma_y: sum_train (y - eta)^2 / sigma_y^2 - n_train + prior
    g = v - m.ntrain[fold_of_chain(m, c)] + prior_grad(m, m.q1[idx], j);
  } else {
    const double u = uscr[c];
    const double tau = exp(u);
    g = j == m.p + 1 ? tau * v + prior_grad(m, u, j) : tau * v - m.q1[idx];
  }
  if (mode == 0) m.g1[idx] = g;
  else leapfrog_update(m, c, j, g, mode == 2);
}

// ----------------------------------------------------------------------------
// Host-side dispatch
// ----------------------------------------------------------------------------
size_t valu_smem_bytes(bool fp64, int W, int family, int n_groups, int pb) {
  const size_t tsz = fp64 ? 8 : 4;
  const size_t jc = std::min<size_t>(fp64 ? 4 : 8, static_cast<size_t>(pb));
  size_t b = tsz * W * jc * 64 + 8 * W * 64;
  b += tsz * static_cast<size_t>(pb) * 64;   // gfin
  if (hier_family(family)) b += 2 * tsz * n_groups * 64 + 2 * tsz * W * 64 + 8 * W;   // zt, rg, edge slots
  return b;
}

int valu_pb(int64_t p, bool fp64) {
  if (p <= 4) return 4;
  if (p <= 8) return 8;
  if (p <= 16) return 16;
  if (p <= 32) return 32;
  if (p <= 64) return 64;
  (void)fp64;
  return 0;
}
#endif

template <typename T, int FAM, int PB>
static hipError_t launch_mode(const ValuArgs& a, int W, hipStream_t st, size_t smem, int nblk, int ns = 1) {
  dim3 grid(nblk), block(64 * W);
  if (a.mode == MODE_PART) {
    hipLaunchKernelGGL((k_valu_part<T, FAM, PB>), dim3(nblk, ns), block, smem, st, a);
    return hipGetLastError();
  }
  if (a.mode == MODE_GRAD) hipLaunchKernelGGL((k_valu_grad<T, FAM, PB>), grid, block, smem, st, a);
  else if (a.mode == MODE_LEAP) hipLaunchKernelGGL((k_valu_leap<T, FAM, PB>), grid, block, smem, st, a);
  else hipLaunchKernelGGL((k_valu_iter<T, FAM, PB>), grid, block, smem, st, a);
  return hipGetLastError();
}

template <typename T, int FAM>
hipError_t launch_fam(const ValuArgs& a, int pb, int W, hipStream_t st, size_t smem, int nblk, int ns) {
  switch (pb) {
    case 4: return launch_mode<T, FAM, 4>(a, W, st, smem, nblk, ns);
    case 8: return launch_mode<T, FAM, 8>(a, W, st, smem, nblk, ns);
    case 16: return launch_mode<T, FAM, 16>(a, W, st, smem, nblk, ns);
    case 32: return launch_mode<T, FAM, 32>(a, W, st, smem, nblk, ns);
    case 64: return launch_mode<T, FAM, 64>(a, W, st, smem, nblk, ns);
  }
  return hipErrorInvalidValue;
}

// Workgroups of k_valu_part per compute unit (registers, LDS and threads),
// from the runtime's occupancy calculator; 0 if unknown.
template <typename T, int FAM>
int part_occupancy_fam(int pb, int W, size_t smem) {
  const void* f = nullptr;
  switch (pb) {
    case 4: f = reinterpret_cast<const void*>(&k_valu_part<T, FAM, 4>); break;
    case 8: f = reinterpret_cast<const void*>(&k_valu_part<T, FAM, 8>); break;
    case 16: f = reinterpret_cast<const void*>(&k_valu_part<T, FAM, 16>); break;
    case 32: f = reinterpret_cast<const void*>(&k_valu_part<T, FAM, 32>); break;
    case 64: f = reinterpret_cast<const void*>(&k_valu_part<T, FAM, 64>); break;
  }
  int nb = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * W, smem) != hipSuccess) return 0;
  return nb;
}

#if defined(PCV_VALU_T)
// This translation unit instantiates the kernels of one (arithmetic type,
// family) pair; the build compiles the file once per pair, in parallel.
template hipError_t launch_fam<PCV_VALU_T, PCV_VALU_FAM>(const ValuArgs&, int, int, hipStream_t, size_t, int, int);
template int part_occupancy_fam<PCV_VALU_T, PCV_VALU_FAM>(int, int, size_t);
}  // namespace pcv
#else
#define PCV_VALU_EXTERN(T, F)                                                                                 \
  extern template hipError_t launch_fam<T, F>(const ValuArgs&, int, int, hipStream_t, size_t, int, int); \
  extern template int part_occupancy_fam<T, F>(int, int, size_t);
PCV_VALU_EXTERN(double, FAM_GAUSS)
PCV_VALU_EXTERN(double, FAM_LOGIT)
PCV_VALU_EXTERN(double, FAM_POIS)
PCV_VALU_EXTERN(double, FAM_HIER)
PCV_VALU_EXTERN(double, FAM_HGAUSS)
PCV_VALU_EXTERN(float, FAM_GAUSS)
PCV_VALU_EXTERN(float, FAM_LOGIT)
PCV_VALU_EXTERN(float, FAM_POIS)
PCV_VALU_EXTERN(float, FAM_HIER)
PCV_VALU_EXTERN(float, FAM_HGAUSS)
#undef PCV_VALU_EXTERN

hipError_t launch_valu(const DevModel& m, const void* Xv, bool fp64, int pb, int W, int mode, int64_t t0,
                       int n_iter, int n_steps, hipStream_t st) {
  ValuArgs a;
  a.m = m;
  a.Xv = Xv;
  a.t0 = t0;
  a.n_iter = n_iter;
  a.mode = mode;
  a.n_steps = n_steps;
  const int nblk = static_cast<int>((m.C + 63) / 64);
  const size_t smem = valu_smem_bytes(fp64, W, m.family, m.n_groups, pb);
  if (fp64) {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<double, FAM_GAUSS>(a, pb, W, st, smem, nblk, 1);
      case FAM_LOGIT: return launch_fam<double, FAM_LOGIT>(a, pb, W, st, smem, nblk, 1);
      case FAM_POIS: return launch_fam<double, FAM_POIS>(a, pb, W, st, smem, nblk, 1);
      case FAM_HIER: return launch_fam<double, FAM_HIER>(a, pb, W, st, smem, nblk, 1);
      case FAM_HGAUSS: return launch_fam<double, FAM_HGAUSS>(a, pb, W, st, smem, nblk, 1);
    }
  } else {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<float, FAM_GAUSS>(a, pb, W, st, smem, nblk, 1);
      case FAM_LOGIT: return launch_fam<float, FAM_LOGIT>(a, pb, W, st, smem, nblk, 1);
      case FAM_POIS: return launch_fam<float, FAM_POIS>(a, pb, W, st, smem, nblk, 1);
      case FAM_HIER: return launch_fam<float, FAM_HIER>(a, pb, W, st, smem, nblk, 1);
      case FAM_HGAUSS: return launch_fam<float, FAM_HGAUSS>(a, pb, W, st, smem, nblk, 1);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_valu_part(const DevModel& m, const void* Xv, bool fp64, int pb, int W, int ns, double* Gpart,
                            double* Vpart, double* uscr, bool value, bool series, hipStream_t st) {
  ValuArgs a{};
  a.m = m;
  a.Xv = Xv;
  a.mode = MODE_PART;
  a.Gpart = Gpart;
  a.Vpart = Vpart;
  a.uscr = uscr;
  a.value = value ? 1 : 0;
  a.series = series && !hier_family(m.family) ? 1 : 0;
  const int nblk = static_cast<int>((m.C + 63) / 64);
  const size_t smem = valu_smem_bytes(fp64, W, m.family, m.n_groups, pb);
  if (fp64) {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<double, FAM_GAUSS>(a, pb, W, st, smem, nblk, ns);
      case FAM_LOGIT: return launch_fam<double, FAM_LOGIT>(a, pb, W, st, smem, nblk, ns);
      case FAM_POIS: return launch_fam<double, FAM_POIS>(a, pb, W, st, smem, nblk, ns);
      case FAM_HIER: return launch_fam<double, FAM_HIER>(a, pb, W, st, smem, nblk, ns);
      case FAM_HGAUSS: return launch_fam<double, FAM_HGAUSS>(a, pb, W, st, smem, nblk, ns);
    }
  } else {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<float, FAM_GAUSS>(a, pb, W, st, smem, nblk, ns);
      case FAM_LOGIT: return launch_fam<float, FAM_LOGIT>(a, pb, W, st, smem, nblk, ns);
      case FAM_POIS: return launch_fam<float, FAM_POIS>(a, pb, W, st, smem, nblk, ns);
      case FAM_HIER: return launch_fam<float, FAM_HIER>(a, pb, W, st, smem, nblk, ns);
      case FAM_HGAUSS: return launch_fam<float, FAM_HGAUSS>(a, pb, W, st, smem, nblk, ns);
    }
  }
  return hipErrorInvalidValue;
}

int valu_part_occupancy(bool fp64, int family, int pb, int W, size_t smem) {
  switch (family) {
    case FAM_GAUSS: return fp64 ? part_occupancy_fam<double, FAM_GAUSS>(pb, W, smem) : part_occupancy_fam<float, FAM_GAUSS>(pb, W, smem);
    case FAM_LOGIT: return fp64 ? part_occupancy_fam<double, FAM_LOGIT>(pb, W, smem) : part_occupancy_fam<float, FAM_LOGIT>(pb, W, smem);
    case FAM_POIS: return fp64 ? part_occupancy_fam<double, FAM_POIS>(pb, W, smem) : part_occupancy_fam<float, FAM_POIS>(pb, W, smem);
    case FAM_HIER: return fp64 ? part_occupancy_fam<double, FAM_HIER>(pb, W, smem) : part_occupancy_fam<float, FAM_HIER>(pb, W, smem);
    case FAM_HGAUSS: return fp64 ? part_occupancy_fam<double, FAM_HGAUSS>(pb, W, smem) : part_occupancy_fam<float, FAM_HGAUSS>(pb, W, smem);
  }
  return 0;
}

hipError_t launch_valu_finish(const DevModel& m, const double* Gpart, const double* uscr, int ns, int mode,
                              hipStream_t st) {
  if (!hier_family(m.family)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_valu_finish, dim3(static_cast<unsigned>((m.d * m.C + 255) / 256)), dim3(256), 0, st, m, Gpart,
                     uscr, ns, mode);
  return hipGetLastError();
}

}  // namespace pcv
#endif
