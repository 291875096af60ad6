// Fused VALU path: one workgroup owns 64 chains (one per lane) and runs whole
// HMC transitions for them -- momentum, S masked value/gradient evaluations
// with the leapfrog updates, Metropolis test, log predictive and
// accumulation -- without any grid-wide synchronisation, because chains never
// interact (Section 3.3).  The W waves of the workgroup split the rows; each
// row of X is read once per wave with scalar loads and broadcast to the 64
// chains.  Used for narrow designs (p <= 32 in fp64, p <= 64 in fp32).
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
template <typename T, int FAM, int PB, bool VALUE>
__device__ __forceinline__ void grad_eval(const DevModel& m, const T* __restrict__ Xv, int lane, int wave,
                                          int W, int64_t cc, int k, int elo, int ehi, T (&G)[PB],
                                          double& val, char* smem, bool want_value = true,
                                          const int32_t* wave_rows = nullptr) {
  constexpr int JC = sizeof(T) == 8 ? 4 : 8;
  T* red = reinterpret_cast<T*>(smem);                                      // [W][JC][64]
  double* vred = reinterpret_cast<double*>(smem + sizeof(T) * W * JC * 64);  // [W][64]
  T* zt = reinterpret_cast<T*>(smem + sizeof(T) * W * JC * 64 + sizeof(double) * W * 64);  // [G][64]
  T* rg = zt + (FAM == FAM_HIER ? m.n_groups * 64 : 0);                      // [G][64]
  T* gfin = rg + (FAM == FAM_HIER ? m.n_groups * 64 : 0);                    // [PB][64]

  T th[PB];
#pragma unroll
  for (int j = 0; j < PB; ++j) th[j] = (j < m.p) ? static_cast<T>(m.q1[j * m.C + cc]) : T(0);
  T mu = 0;
  if (FAM == FAM_HIER) {
    mu = static_cast<T>(m.q1[m.p * m.C + cc]);
    const T tau = static_cast<T>(exp(m.q1[(m.p + 1) * m.C + cc]));
    for (int g = wave; g < m.n_groups; g += W) {
      zt[g * 64 + lane] = tau * static_cast<T>(m.q1[(m.p + 2 + g) * m.C + cc]);
      rg[g * 64 + lane] = T(0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < PB; ++j) G[j] = T(0);
  val = 0.0;
  const T is2 = static_cast<T>(m.inv_sigma2);
  const int32_t* wr = wave_rows ? wave_rows : m.wave_rows;
  const int64_t r0 = wr[wave], r1 = wr[wave + 1];
  int gcur = -1;
  T racc = T(0);
  for (int64_t i = r0; i < r1; ++i) {
    const T* xr = Xv + i * PB;
    T xv[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) xv[j] = xr[j];
    T eta = T(0);
#pragma unroll
    for (int j = 0; j < PB; ++j) eta += xv[j] * th[j];
    if (FAM == FAM_HIER) {
      const int g = m.group_of[i];
      if (g != gcur) {
        if (gcur >= 0) rg[gcur * 64 + lane] += racc;
        gcur = g;
        racc = T(0);
      }
      eta += mu + zt[g * 64 + lane];
    }
    bool train;
    if (m.fold_kind == PCV_FOLDS_INDEX) train = m.fold_index[i] != k;
    else if (m.fold_kind == PCV_FOLDS_INTERVALS) train = (i < elo) || (i >= ehi);
    else train = m.roles[static_cast<int64_t>(k) * m.n + i] == 1;
    const T y = ValuY<T>::get(m, i);
    const T r = train ? vresid<FAM, T>(y, eta, is2) : T(0);
#pragma unroll
    for (int j = 0; j < PB; ++j) G[j] += xv[j] * r;
    if (FAM == FAM_HIER) racc += r;
    if (VALUE && want_value) {
      if (train) val += static_cast<double>(vell0<FAM, T>(y, eta, is2));
    }
  }
  if (FAM == FAM_HIER && gcur >= 0) rg[gcur * 64 + lane] += racc;

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
}

// Wave 0, lane = chain: add the prior to the reduced likelihood gradient
// (LDS gfin) and hand the full gradient to `emit(j, g)`.  The coordinate loop
// is deliberately not unrolled: unrolling hoists one address per coordinate
// out of the leapfrog loop and exhausts the register file.
template <typename T, int FAM, int PB, typename Emit>
__device__ __forceinline__ void finish_chain(const DevModel& m, int64_t c, int lane, char* smem, int W, Emit emit) {
  constexpr int JC = sizeof(T) == 8 ? 4 : 8;
  T* zt = reinterpret_cast<T*>(smem + sizeof(T) * W * JC * 64 + sizeof(double) * W * 64);
  T* rg = zt + (FAM == FAM_HIER ? m.n_groups * 64 : 0);
  const T* gfin = rg + (FAM == FAM_HIER ? m.n_groups * 64 : 0);
#pragma nounroll
  for (int64_t j = 0; j < m.p; ++j)
    emit(j, static_cast<double>(gfin[j * 64 + lane]) + prior_grad(m, m.q1[j * m.C + c], j));
  if (FAM == FAM_HIER) {
    const double u = m.q1[(m.p + 1) * m.C + c];
    const double tau = exp(u);
    double gmu = 0.0, gu = 0.0;
#pragma nounroll
    for (int g = 0; g < m.n_groups; ++g) {
      const double rs = static_cast<double>(rg[g * 64 + lane]);
      const double z = m.q1[(m.p + 2 + g) * m.C + c];
      gmu += rs;
      gu += z * rs;
      emit(m.p + 2 + g, tau * rs - z);
    }
    emit(m.p, gmu - m.q1[m.p * m.C + c]);
    emit(m.p + 1, tau * gu + prior_grad(m, u, m.p + 1));
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
  const int k = static_cast<int>(cc / m.L);                                    \
  int elo = 0, ehi = 0;                                                        \
  if (m.fold_kind == PCV_FOLDS_INTERVALS) {                                    \
    elo = m.ivals[4 * k + 2];                                                  \
    ehi = m.ivals[4 * k + 3];                                                  \
  }                                                                            \
  T G[PB];                                                                     \
  double val;                                                                  \
  const bool lead = (wave == 0) && valid;

constexpr int VALU_MAX_THREADS = 512;

// Value and gradient at q1 -> g1, logp1.
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_grad(ValuArgs a) {
  VALU_PROLOGUE
  grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, smem);
  if (lead) {
    finish_chain<T, FAM, PB>(m, c, lane, smem, W, [&](int64_t j, double g) { m.g1[j * m.C + c] = g; });
    m.logp1[c] = val + m.fold_const[k] + prior_quad(m, m.q1, c);
  }
}

// n_steps leapfrog steps from (q1, pm): gradient at the start, first half
// kick and drift, then the steps (used to check single trajectories).
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_leap(ValuArgs a) {
  VALU_PROLOGUE
  grad_eval<T, FAM, PB, false>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, smem);
  if (lead) {
    finish_chain<T, FAM, PB>(m, c, lane, smem, W, [&](int64_t j, double g) {
      const int64_t o = j * m.C + c;
      const double p = m.pm[o] + 0.5 * m.eps * g;
      m.pm[o] = p;
      m.q1[o] += m.eps * m.minv[j] * p;
    });
  }
  __syncthreads();
  for (int s = 0; s < a.n_steps; ++s) {
    const bool last = s == a.n_steps - 1;
    grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, smem);
    if (lead) {
      finish_chain<T, FAM, PB>(m, c, lane, smem, W,
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
      grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, smem, last);
      if (lead) {
        finish_chain<T, FAM, PB>(m, c, lane, smem, W,
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
// split (group-aligned for the hierarchical family).  Wave 0 writes the raw
// partial sums -- sum x r per coefficient and, hierarchical, sum r per group
// -- and the partial value; k_valu_finish adds the splits in a fixed order.
template <typename T, int FAM, int PB>
__global__ __launch_bounds__(VALU_MAX_THREADS) void k_valu_part(ValuArgs a) {
  VALU_PROLOGUE
  const int sp = blockIdx.y;
  const int32_t* wr = m.wave_rows + static_cast<int64_t>(sp) * (W + 1);
  if (a.value) grad_eval<T, FAM, PB, true>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, smem, true, wr);
  else grad_eval<T, FAM, PB, false>(m, Xv, lane, wave, W, cc, k, elo, ehi, G, val, smem, false, wr);
  if (lead) {
    constexpr int JC = sizeof(T) == 8 ? 4 : 8;
    T* zt = reinterpret_cast<T*>(smem + sizeof(T) * W * JC * 64 + sizeof(double) * W * 64);
    const T* rg = zt + (FAM == FAM_HIER ? m.n_groups * 64 : 0);
    const T* gfin = rg + (FAM == FAM_HIER ? m.n_groups * 64 : 0);
    const int64_t R = m.p + (FAM == FAM_HIER ? m.n_groups : 0);
    double* out = a.Gpart + static_cast<int64_t>(sp) * R * m.C + c;
#pragma nounroll
    for (int64_t j = 0; j < m.p; ++j) out[j * m.C] = static_cast<double>(gfin[j * 64 + lane]);
    if (FAM == FAM_HIER) {
#pragma nounroll
      for (int g = 0; g < m.n_groups; ++g) out[(m.p + g) * m.C] = static_cast<double>(rg[g * 64 + lane]);
    }
    if (a.value) a.Vpart[static_cast<int64_t>(sp) * m.C + c] = val;
  }
}

// Sum of the row-split partials over the splits, in a fixed order, one thread
// per (entry, chain), into the first split's slab (in place).
__global__ void k_valu_sum(DevModel m, double* __restrict__ Gpart, int ns, int64_t R) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= R * m.C) return;
  double v = 0.0;
  for (int sp = 0; sp < ns; ++sp) v += Gpart[static_cast<int64_t>(sp) * R * m.C + idx];
  Gpart[idx] = v;
}

// Prior and (hierarchical) the chain rule for mu, log tau and z over the
// summed partials (ns slabs, normally 1 after k_valu_sum); then as k_reduce:
// mode 0 writes g1, 1 and 2 apply a (last) leapfrog update.
template <int FAM>
__global__ void k_valu_finish(DevModel m, const double* __restrict__ Gpart, int ns, int mode) {
  const int64_t c = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (c >= m.C) return;
  const int64_t R = m.p + (FAM == FAM_HIER ? m.n_groups : 0);
  auto total = [&](int64_t j) {
    double v = 0.0;
    for (int sp = 0; sp < ns; ++sp) v += Gpart[(static_cast<int64_t>(sp) * R + j) * m.C + c];
    return v;
  };
  auto emit = [&](int64_t j, double g) {
    if (mode == 0) m.g1[j * m.C + c] = g;
    else leapfrog_update(m, c, j, g, mode == 2);
  };
  for (int64_t j = 0; j < m.p; ++j) emit(j, total(j) + prior_grad(m, m.q1[j * m.C + c], j));
  if (FAM == FAM_HIER) {
    const double u = m.q1[(m.p + 1) * m.C + c];
    const double tau = exp(u);
    double gmu = 0.0, gu = 0.0;
    for (int g = 0; g < m.n_groups; ++g) {
      const double rs = total(m.p + g);
      const double z = m.q1[(m.p + 2 + g) * m.C + c];
      gmu += rs;
      gu += z * rs;
      emit(m.p + 2 + g, tau * rs - z);
    }
    emit(m.p, gmu - m.q1[m.p * m.C + c]);
    emit(m.p + 1, tau * gu + prior_grad(m, u, m.p + 1));
  }
}

// ----------------------------------------------------------------------------
// Host-side dispatch
// ----------------------------------------------------------------------------
size_t valu_smem_bytes(bool fp64, int W, int family, int n_groups) {
  const size_t tsz = fp64 ? 8 : 4;
  const size_t jc = fp64 ? 4 : 8;
  size_t b = tsz * W * jc * 64 + 8 * W * 64;
  if (family == FAM_HIER) b += 2 * tsz * n_groups * 64;
  return b + tsz * 64 * 64;   // gfin, sized for the widest PB
}

int valu_pb(int64_t p, bool fp64) {
  if (p <= 8) return 8;
  if (p <= 16) return 16;
  if (p <= 32) return 32;
  if (!fp64 && p <= 64) return 64;
  return 0;
}

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
static hipError_t launch_fam(const ValuArgs& a, int pb, int W, hipStream_t st, size_t smem, int nblk, int ns = 1) {
  switch (pb) {
    case 8: return launch_mode<T, FAM, 8>(a, W, st, smem, nblk, ns);
    case 16: return launch_mode<T, FAM, 16>(a, W, st, smem, nblk, ns);
    case 32: return launch_mode<T, FAM, 32>(a, W, st, smem, nblk, ns);
    case 64:
      if constexpr (sizeof(T) == 4) return launch_mode<T, FAM, 64>(a, W, st, smem, nblk, ns);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

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
  const size_t smem = valu_smem_bytes(fp64, W, m.family, m.n_groups);
  if (fp64) {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<double, FAM_GAUSS>(a, pb, W, st, smem, nblk);
      case FAM_LOGIT: return launch_fam<double, FAM_LOGIT>(a, pb, W, st, smem, nblk);
      case FAM_POIS: return launch_fam<double, FAM_POIS>(a, pb, W, st, smem, nblk);
      case FAM_HIER: return launch_fam<double, FAM_HIER>(a, pb, W, st, smem, nblk);
    }
  } else {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<float, FAM_GAUSS>(a, pb, W, st, smem, nblk);
      case FAM_LOGIT: return launch_fam<float, FAM_LOGIT>(a, pb, W, st, smem, nblk);
      case FAM_POIS: return launch_fam<float, FAM_POIS>(a, pb, W, st, smem, nblk);
      case FAM_HIER: return launch_fam<float, FAM_HIER>(a, pb, W, st, smem, nblk);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_valu_part(const DevModel& m, const void* Xv, bool fp64, int pb, int W, int ns, double* Gpart,
                            double* Vpart, bool value, hipStream_t st) {
  ValuArgs a{};
  a.m = m;
  a.Xv = Xv;
  a.mode = MODE_PART;
  a.Gpart = Gpart;
  a.Vpart = Vpart;
  a.value = value ? 1 : 0;
  const int nblk = static_cast<int>((m.C + 63) / 64);
  const size_t smem = valu_smem_bytes(fp64, W, m.family, m.n_groups);
  if (fp64) {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<double, FAM_GAUSS>(a, pb, W, st, smem, nblk, ns);
      case FAM_LOGIT: return launch_fam<double, FAM_LOGIT>(a, pb, W, st, smem, nblk, ns);
      case FAM_POIS: return launch_fam<double, FAM_POIS>(a, pb, W, st, smem, nblk, ns);
      case FAM_HIER: return launch_fam<double, FAM_HIER>(a, pb, W, st, smem, nblk, ns);
    }
  } else {
    switch (m.family) {
      case FAM_GAUSS: return launch_fam<float, FAM_GAUSS>(a, pb, W, st, smem, nblk, ns);
      case FAM_LOGIT: return launch_fam<float, FAM_LOGIT>(a, pb, W, st, smem, nblk, ns);
      case FAM_POIS: return launch_fam<float, FAM_POIS>(a, pb, W, st, smem, nblk, ns);
      case FAM_HIER: return launch_fam<float, FAM_HIER>(a, pb, W, st, smem, nblk, ns);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_valu_sum(const DevModel& m, double* Gpart, int ns, hipStream_t st) {
  const int64_t R = m.p + (m.family == FAM_HIER ? m.n_groups : 0);
  hipLaunchKernelGGL(k_valu_sum, dim3(static_cast<unsigned>((R * m.C + 255) / 256)), dim3(256), 0, st, m, Gpart, ns,
                     R);
  return hipGetLastError();
}

hipError_t launch_valu_finish(const DevModel& m, const double* Gpart, int ns, int mode, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((m.C + 255) / 256)), block(256);
  switch (m.family) {
    case FAM_GAUSS: hipLaunchKernelGGL((k_valu_finish<FAM_GAUSS>), grid, block, 0, st, m, Gpart, ns, mode); break;
    case FAM_LOGIT: hipLaunchKernelGGL((k_valu_finish<FAM_LOGIT>), grid, block, 0, st, m, Gpart, ns, mode); break;
    case FAM_POIS: hipLaunchKernelGGL((k_valu_finish<FAM_POIS>), grid, block, 0, st, m, Gpart, ns, mode); break;
    case FAM_HIER: hipLaunchKernelGGL((k_valu_finish<FAM_HIER>), grid, block, 0, st, m, Gpart, ns, mode); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pcv
