// Split-precision MFMA path for wide designs (p = 64 or 128).
//
// One gradient evaluation of all C chains is
//     eta = X Theta   ->  r = mask * dl/deta  ->  G = X' R        (Appendix B)
// with X [n,p] shared by every chain.  Both contractions run on the bf16
// matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16) with fp32 accumulation;
// precision is won back by splitting operands into bf16 terms:
//   X      = Xhi + Xlo exactly (the stored design)
//   Theta ~= t0 + t1 (+ t2): two terms (FWD=3 products) or three (FWD=5)
//   R     ~= Rhi + Rlo
//   eta = Xhi t0 + Xhi t1 + Xlo t0 [+ Xhi t2 + Xlo t1],  G = Xhi' Rhi + Xhi' Rlo + Xlo' Rhi
// eta is never written to memory: the forward accumulator of a 32-row tile
// is turned into the residual in registers and fed straight back as the
// B operand of the adjoint product.  The row order of the adjoint's K
// dimension is permuted to match the accumulator layout, and X is stored
// pre-packed in both fragment orders so each wave reads its operands from
// LDS with one 16-byte load per lane.
//
// Work split: a workgroup (8 waves x 32 chains = 256 chains) takes one chain
// tile and one contiguous range of row tiles ("split"); its partial G and
// partial log likelihood go to a buffer that k_reduce sums in a fixed order.
#include "pcv_internal.h"

namespace pcv {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MF_WAVES = 8;
constexpr int MF_CHAINS_PER_WAVE = 32;
constexpr int MF_CHAIN_TILE = MF_WAVES * MF_CHAINS_PER_WAVE;  // 256
constexpr int MF_ROWS = 32;                                   // rows per tile

// The kernels' design width P: p rounded up to 64 or 128.  X is packed with
// zero columns past p, theta is taken as zero there, and only the first p
// gradient rows are written, so any 1 <= p <= 128 runs on the P kernels.
int mfma_width(int64_t p) { return p <= 64 ? 64 : 128; }
int mfma_chain_tile(int shape);
int mfma_layout(int shape);

// fragments per 32-row tile: forward 2 (M) x P/32 (K) x 2 planes, adjoint P/16 (M) x 2 planes
__host__ __device__ constexpr int mf_nfrag_fwd(int P) { return 2 * (P / 32) * 2; }
__host__ __device__ constexpr int mf_nfrag(int P) { return mf_nfrag_fwd(P) + (P / 16) * 2; }

struct MfmaArgs {
  DevModel m;
  const uint4* Xpk;    // [n_tiles][nfrag][64] x 16 B
  const float* ty;     // [n_tiles*32] y per (padded) row
  const int32_t* tfid; // [n_tiles*32] fold index per row (INDEX encoding)
  float* Gpart;        // [n_splits][P][C]
  double* Vpart;       // [n_splits][C]
  const uint32_t* tflag;  // [n_tiles][chain tiles]: bit w = wave w sees a non-train or padded row
  int n_tiles, tiles_per_split, n_splits;
};

constexpr int MF_XCDS = 8;
// Bijection on [0, nb): the workgroups of XCD x (b % 8 == x, in launch order
// b / 8) get tasks x*per + min(x, rem) + b/8, a contiguous range per XCD.
__host__ __device__ constexpr int mf_xcd_task(int b, int nb) {
  const int per = nb / MF_XCDS, rem = nb % MF_XCDS;
  const int x = b % MF_XCDS;
  return x * per + (x < rem ? x : rem) + b / MF_XCDS;
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }

// Residual dl/deta and (optionally) l(y, eta) without its row constant, in
// fp32 with hardware exp/log/rcp (errors ~1e-7 relative, far below the bf16
// split error of eta itself).
// For the logistic and Poisson families the forward product returns
// e2 = eta * log2(e) (theta is scaled by log2(e) when it is split), so the
// exponentials are single v_exp_f32 (base 2) instructions.
constexpr float LOG2E_F = 1.4426950408889634f;
constexpr double LOG2E_D = 1.4426950408889634;
constexpr float LN2_F = 0.6931471805599453f;
template <int FAM>
__host__ __device__ constexpr double mf_theta_scale() { return FAM == FAM_GAUSS ? 1.0 : LOG2E_D; }
template <int FAM>
__device__ __forceinline__ float mf_resid(float y, float e2, float is2) {
  if (FAM == FAM_GAUSS) return (y - e2) * is2;
  if (FAM == FAM_POIS) return y - __builtin_amdgcn_exp2f(e2);
  return y - __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-e2));
}

// Value launches need the residual and the log-likelihood of the same
// element; one exponential serves both (logistic: t = e^{-|eta|} gives
// sigma(eta) = (eta >= 0 ? 1 : t) / (1 + t) and log(1 + t) from the same
// 1 + t; Poisson: the mean; Gaussian: the difference y - eta).  The
// logistic l0 is returned in base-2 units (l0 / ln 2: the logarithm is the
// hardware's log2 and e2 = eta log2 e already); mf_ell0_scale gives the
// factor the launch applies to its per-chain sums.  log2 of the rounded
// 1 + t loses at most one ulp of 1 (below 2e-7) where t is tiny, against
// terms of order 1.
template <int FAM>
__host__ __device__ constexpr double mf_ell0_scale() { return FAM == FAM_LOGIT ? 0.6931471805599453 : 1.0; }
template <int FAM>
__device__ __forceinline__ void mf_resid_ell0(float y, float e2, float is2, float& r, float& l0) {
  if (FAM == FAM_GAUSS) {
    const float d = y - e2;
    r = d * is2;
    l0 = -0.5f * d * r;
  } else if (FAM == FAM_POIS) {
    const float lam = __builtin_amdgcn_exp2f(e2);
    r = y - lam;
    l0 = y * (e2 * LN2_F) - lam;
  } else {
    const float t = __builtin_amdgcn_exp2f(-fabsf(e2));    // e^{-|eta|} in (0, 1]
    const float q = 1.0f + t;
    r = y - (e2 >= 0.0f ? 1.0f : t) * __builtin_amdgcn_rcpf(q);
    l0 = y * e2 - fmaxf(e2, 0.0f) - __builtin_amdgcn_logf(q);   // base 2
  }
}

// theta[j][c] at the 8 KB coordinates j = KS kb + off + e (kb < KB, e < 8)
// of chain c, split into NT bf16 terms (the MFMA B operand; pre-scaled by
// log2 e for the logistic and Poisson families).  Coordinates past p (the
// design's zero columns up to the kernel's width) and coordinates a nested
// model drops take theta = 0.  Every load is unconditional, from a clamped
// chain and coordinate, and the selection comes after: a guarded load would
// become a branch with a wait of its own, and the lane's loads would run
// one round trip at a time instead of all in flight together.
template <int FAM, int NT, int KB, int KS, bool MASKED>
__device__ __forceinline__ void mf_theta_terms(const DevModel& m, int64_t c, int off, bf16x8 (&out)[NT][KB]) {
  const bool cv = c < m.C;
  const int64_t cc = cv ? c : m.C - 1;
  const uint8_t* mrow = MASKED ? mask_row(m, cc) : nullptr;
  double tv[KB][8];
  bool keep[KB][8];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = KS * kb + off + e;
      const int jc = j < m.p ? j : static_cast<int>(m.p) - 1;
      tv[kb][e] = m.q1[static_cast<int64_t>(jc) * m.C + cc];
      const uint8_t mb = MASKED ? mrow[jc] : 1;
      keep[kb][e] = cv & (j < m.p) & (mb != 0);
    }
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const double t = keep[kb][e] ? tv[kb][e] * mf_theta_scale<FAM>() : 0.0;
      if (NT == 2) {
        const float t32 = static_cast<float>(t);
        const __bf16 h = to_bf16(t32);
        out[0][kb][e] = h;
        out[1][kb][e] = to_bf16(t32 - static_cast<float>(h));
      } else {
        const __bf16 h = to_bf16(static_cast<float>(t));
        const double r1 = t - static_cast<double>(static_cast<float>(h));
        const __bf16 mdl = to_bf16(static_cast<float>(r1));
        const double r2 = r1 - static_cast<double>(static_cast<float>(mdl));
        out[0][kb][e] = h;
        out[1][kb][e] = mdl;
        out[NT - 1][kb][e] = to_bf16(static_cast<float>(r2));
      }
    }
}

// CB = 16-chain blocks per wave: 2 (32 chains per wave, 256 per workgroup,
// one workgroup per CU) or 1 (16 chains per wave, 128 per workgroup; at
// P = 64 the registers then fit two workgroups per CU, four waves per SIMD,
// at the cost of twice the fragment reads per MFMA).
template <int FAM, int P, int FWD, bool VALUE, int FK, int CB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(CB == 1 ? 4 : 1))) void k_mfma(MfmaArgs a) {
  static_assert(CB == 2 || (CB == 1 && P == 64), "16 chains per wave only at width 64");
  constexpr int CPW = 16 * CB;                    // chains per wave
  constexpr int CT = MF_WAVES * CPW;              // chains per workgroup
  constexpr int KB = P / 32;
  constexpr int MB = P / 16;
  constexpr int NFF = mf_nfrag_fwd(P);
  constexpr int NF = mf_nfrag(P);
  constexpr int NST = NF * 64 / (64 * MF_WAVES);  // uint4 staged per thread
  constexpr int NT = FWD == 5 ? 3 : 2;             // theta terms
  constexpr int NBUF = 4;                          // LDS ring of row tiles
  static_assert(NST * 64 * MF_WAVES == NF * 64, "staging must tile the fragments");
  static_assert(NST == 2 || NST == 4, "two or four staged vectors per thread");

  __shared__ __align__(16) uint4 sfrag[NBUF][NF * 64];
  __shared__ float sy[NBUF][MF_ROWS];
  __shared__ int32_t sf[NBUF][MF_ROWS];

  const DevModel& m = a.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g4 = lane >> 4;
  const int l16 = lane & 15;
  // Workgroups are dealt round-robin to the 8 XCDs (workgroup b runs on XCD
  // b % 8).  Renumber so each XCD gets a contiguous range of tasks, and order
  // tasks split-major: the workgroups resident on one XCD then share a row
  // split and stream the same X tiles through that XCD's L2 together.
  const int task = mf_xcd_task(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int n_ct = static_cast<int>((m.C + CT - 1) / CT);
  const int sp = task / n_ct;
  const int ct = task - sp * n_ct;
  const int64_t cbase = static_cast<int64_t>(ct) * CT + wave * CPW;
  const bool wave_active = cbase < m.C;
  const int t_beg = sp * a.tiles_per_split;
  const int t_end = min(a.n_tiles, t_beg + a.tiles_per_split);
  const int t_last = t_end > t_beg ? t_end - 1 : t_beg;

  // chains of this lane in its CB 16-chain blocks
  int kf[CB], elo[CB], ehi[CB];
  int64_t cidx[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int64_t c = cbase + cb * 16 + l16;
    cidx[cb] = c;
    const int64_t cc = c < m.C ? c : m.C - 1;
    kf[cb] = fold_of_chain(m, cc);
    elo[cb] = 0;
    ehi[cb] = 0;
    if (FK == PCV_FOLDS_INTERVALS) {
      elo[cb] = m.ivals[4 * kf[cb] + 2];
      ehi[cb] = m.ivals[4 * kf[cb] + 3];
    }
  }

  // theta operand fragments: lane holds theta[k = kb*32 + 8*g4 + e][chain]
  bf16x8 th[NT][KB][CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    bf16x8 t[NT][KB];
    if (m.mmask) mf_theta_terms<FAM, NT, KB, 32, true>(m, cidx[cb], 8 * g4, t);
    else mf_theta_terms<FAM, NT, KB, 32, false>(m, cidx[cb], 8 * g4, t);
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) th[q][kb][cb] = t[q][kb];
  }

  f32x4 gacc[MB][CB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) gacc[mb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  double vacc[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) vacc[cb] = 0.0;
  const float is2 = static_cast<float>(m.inv_sigma2);
  const int nrows = static_cast<int>(m.n);

  // ---- staging: global -> registers -> LDS ring ---------------------------
  uint4 st0, st1, st2, st3;   // named registers: a private array here ends up in scratch
  float my_y = 0.f;
  int32_t my_f = 0;
  auto load_stage = [&](int tt) {
    const uint4* src = a.Xpk + static_cast<int64_t>(tt) * NF * 64;
    st0 = src[tid];
    st1 = src[512 + tid];
    if constexpr (NST == 4) {
      st2 = src[1024 + tid];
      st3 = src[1536 + tid];
    }
    // every thread carries the metadata of row (tid mod 32): duplicate stores
    // of equal values keep the loop body free of branches
    my_y = a.ty[static_cast<int64_t>(tt) * MF_ROWS + (tid & (MF_ROWS - 1))];
    my_f = a.tfid[static_cast<int64_t>(tt) * MF_ROWS + (tid & (MF_ROWS - 1))];
  };
  auto store_stage = [&](int b) {
    sfrag[b][tid] = st0;
    sfrag[b][512 + tid] = st1;
    if constexpr (NST == 4) {
      sfrag[b][1024 + tid] = st2;
      sfrag[b][1536 + tid] = st3;
    }
    sy[b][tid & (MF_ROWS - 1)] = my_y;
    sf[b][tid & (MF_ROWS - 1)] = my_f;
  };

  // forward product of one tile (buffer b): eta[32 rows x CPW chains]
  auto forward = [&](int b, f32x4 (&eta)[2][CB]) {
#pragma unroll
    for (int mh = 0; mh < 2; ++mh)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) eta[mh][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int mh = 0; mh < 2; ++mh) {
        const int f = (mh * KB + kb) * 2;
        const bf16x8 x0 = __builtin_bit_cast(bf16x8, sfrag[b][f * 64 + lane]);
        const bf16x8 x1 = __builtin_bit_cast(bf16x8, sfrag[b][(f + 1) * 64 + lane]);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          f32x4 acc = eta[mh][cb];
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, th[0][kb][cb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, th[1][kb][cb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, th[0][kb][cb], acc, 0, 0, 0);
          if (NT == 3) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, th[NT - 1][kb][cb], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, th[1][kb][cb], acc, 0, 0, 0);
          }
          eta[mh][cb] = acc;
        }
      }
    }
  };

  // The per-tile work is cut into NG groups that alternate between the
  // forward product of the next tile (group 2q: K block q/2.. of M half) and
  // the adjoint product of the previous tile (group 2q+1: M block q), each
  // group = two fragment reads + 3 CB (or 5 CB) MFMAs, with EPG epilogue
  // elements of the current tile in between.  The three streams are
  // independent, so the order is pinned with scheduling barriers.
  constexpr int NG = 2 * MB;            // = 2 * (2 * KB)
  constexpr int EPG = 8 * CB / NG;      // epilogue elements per group
  static_assert(EPG * NG == 8 * CB, "8 CB epilogue elements per lane per tile");

  auto frag = [&](int b, int f) { return __builtin_bit_cast(bf16x8, sfrag[b][f * 64 + lane]); };
  auto group_frag_index = [&](int g) {
    // forward groups (even g): (mh, kb) = ((g/2) / KB, (g/2) % KB); adjoint groups (odd g): mb = g/2
    return (g & 1) ? NFF + (g >> 1) * 2 : (((g >> 1) / KB) * KB + ((g >> 1) % KB)) * 2;
  };

  // Skewed software pipeline over row tiles: iteration tt issues
  // forward(tt+1), adjoint(tt-1) and epilogue(tt).  Ring slot of tile tt is
  // (tt - t_beg) mod 4: slots hold tt-1, tt, tt+1 and receive tt+2.
  // Prologue: tile t_beg into slots 0 and 3 (slot 3 stands in for "tile
  // t_beg-1", whose adjoint runs with zero residuals), t_beg+1 into slot 1.
  load_stage(t_beg < t_last ? t_beg : t_last);
  store_stage(0);
  store_stage(3);
  load_stage(min(t_beg + 1, t_last));
  store_stage(1);
  load_stage(min(t_beg + 2, t_last));
  __syncthreads();
  f32x4 eta_cur[2][CB], eta_nxt[2][CB];
  forward(0, eta_cur);
  bf16x8 rph[CB], rpl[CB], rch[CB], rcl[CB];   // residual fragments: previous / current tile
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      rph[cb][e] = to_bf16(0.f);
      rpl[cb][e] = to_bf16(0.f);
    }
  }

  for (int tt = t_beg; tt < t_end; ++tt) {
    const int i = tt - t_beg;
    const int bc = i & 3, b1 = (i + 1) & 3, b2 = (i + 2) & 3, bp = (i + 3) & 3;
    // all waves are done with iteration tt-1; tile tt+1 (stored then) is visible
    __syncthreads();
    store_stage(b2);
    load_stage(min(tt + 3, t_last));
    // (a wave whose chains are all past C computes on clamped chains and
    // discards the result: no branch in the loop body)

    // metadata of the 8 rows this lane sees in tile tt
    float yr[8];
    int fr8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int rl = (e >> 2) * 16 + 4 * g4 + (e & 3);
      yr[e] = sy[bc][rl];
      fr8[e] = sf[bc][rl];
    }
#pragma unroll
    for (int mh = 0; mh < 2; ++mh)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) eta_nxt[mh][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float vt[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) vt[cb] = 0.f;

    bf16x8 xa0 = frag(b1, group_frag_index(0)), xa1 = frag(b1, group_frag_index(0) + 1);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      // prefetch the next group's fragments
      bf16x8 xb0 = xa0, xb1 = xa1;
      if (g + 1 < NG) {
        const int bn = ((g + 1) & 1) ? bp : b1;
        xb0 = frag(bn, group_frag_index(g + 1));
        xb1 = frag(bn, group_frag_index(g + 1) + 1);
      }
      if ((g & 1) == 0) {
        const int q = g >> 1, mh = q / KB, kb = q % KB;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          f32x4 acc = eta_nxt[mh][cb];
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa0, th[0][kb][cb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa0, th[1][kb][cb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa1, th[0][kb][cb], acc, 0, 0, 0);
          if (NT == 3) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa0, th[NT - 1][kb][cb], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa1, th[1][kb][cb], acc, 0, 0, 0);
          }
          eta_nxt[mh][cb] = acc;
        }
      } else {
        const int mb = g >> 1;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          f32x4 acc = gacc[mb][cb];
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa0, rph[cb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa0, rpl[cb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa1, rph[cb], acc, 0, 0, 0);
          gacc[mb][cb] = acc;
        }
      }
      // epilogue elements of tile tt: element index el -> (row slot e, chain block cb)
#pragma unroll
      for (int u = 0; u < EPG; ++u) {
        const int el = g * EPG + u;
        const int e = el / CB, cb = el % CB;
        const int mh = e >> 2, ii = e & 3;
        const int row = tt * MF_ROWS + mh * 16 + 4 * g4 + ii;
        // padded rows (row >= n) hold X = 0, so they add nothing to G; only
        // the value needs them masked
        const bool rv = !VALUE || row < nrows;
        bool train;
        if (FK == PCV_FOLDS_INDEX) train = rv & (fr8[e] != kf[cb]);
        else train = rv & ((row < elo[cb]) | (row >= ehi[cb]));
        const float x = eta_cur[mh][cb][ii];
        float rr, l0 = 0.f;
        if (VALUE) mf_resid_ell0<FAM>(yr[e], x, is2, rr, l0);
        else rr = mf_resid<FAM>(yr[e], x, is2);
        const float r = train ? rr : 0.f;
        if (VALUE) vt[cb] += train ? l0 : 0.f;
        const __bf16 h = to_bf16(r);
        rch[cb][e] = h;
        rcl[cb][e] = to_bf16(r - static_cast<float>(h));
      }
      __builtin_amdgcn_sched_barrier(0);
      xa0 = xb0;
      xa1 = xb1;
    }
    if (VALUE) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) vacc[cb] += static_cast<double>(vt[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      rph[cb] = rch[cb];
      rpl[cb] = rcl[cb];
    }
#pragma unroll
    for (int mh = 0; mh < 2; ++mh)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) eta_cur[mh][cb] = eta_nxt[mh][cb];
  }
  // adjoint of the last tile (its slot is untouched since it was loaded)
  {
    const int bl = (t_end - 1 - t_beg) & 3;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const bf16x8 x0 = frag(bl, NFF + mb * 2), x1 = frag(bl, NFF + mb * 2 + 1);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        f32x4 acc = gacc[mb][cb];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, rph[cb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, rpl[cb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, rph[cb], acc, 0, 0, 0);
        gacc[mb][cb] = acc;
      }
    }
  }

  if (!wave_active) return;
  // ---- partial results -----------------------------------------------------
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int64_t c = cidx[cb];
    if (c < m.C) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int j = mb * 16 + 4 * g4 + ii;
          if (j < m.p) a.Gpart[(static_cast<int64_t>(sp) * m.p + j) * m.C + c] = gacc[mb][cb][ii];
        }
    }
    if (VALUE) {
      double v = vacc[cb];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16 && c < m.C) a.Vpart[static_cast<int64_t>(sp) * m.C + c] = v * mf_ell0_scale<FAM>();
    }
  }
}

// ---------------------------------------------------------------------------
// 32x32x16 variant.  The same product as k_mfma on v_mfma_f32_32x32x16_bf16:
// a wave owns 32 chains (one 32-wide N block) and a 32-row tile is one M
// block, so each MFMA does twice the work of a 16x16x32 one and the matrix
// cores need half the issue slots, which the epilogue's VALU work can use.
// The D layout of a 32x32 accumulator (lane l, element i: row
// 8(i/4) + 4(l/32) + i%4, column l%32) gives each lane 16 rows of ONE chain.
// The adjoint's K index (rows) follows that layout: K half kh, lane half h,
// element e is row 16 kh + (e < 4 ? 4h + e : 8 + 4h + e - 4), so the
// residuals of accumulator elements 8kh..8kh+7 are the adjoint's B operand
// for K half kh as they stand.
//
// Masks leave the per-element path: a per-(tile, chain tile) word, built on
// the host from the fold encoding, has bit w set when some chain of wave w
// has a non-train row in the tile (or the tile has padded rows).  Waves whose
// bit is clear (all but a few tiles: a fold's non-train rows are a small
// fraction of n) take an epilogue without any mask arithmetic.
// ---------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// fragments per 32-row tile: forward P/16 K blocks x 2 planes; adjoint
// P/32 M blocks x 2 K halves x 2 planes
__host__ __device__ constexpr int m2_nfrag_fwd(int P) { return (P / 16) * 2; }
__host__ __device__ constexpr int m2_nfrag(int P) { return m2_nfrag_fwd(P) + (P / 32) * 4; }

// Row (within the tile) of accumulator element i for lane half h.
__host__ __device__ constexpr int m2_row(int i, int h) { return 8 * (i >> 2) + 4 * h + (i & 3); }

// The pair (r0, r1) as packed bf16 hi and lo words: hi = bf16(r) (round to
// nearest even, v_cvt_pk_bf16_f32), lo = bf16(r - hi).
__device__ __forceinline__ void m2_split2(float r0, float r1, uint32_t& hi, uint32_t& lo) {
  const bf16x2 h = __builtin_convertvector(f32x2{r0, r1}, bf16x2);
  const uint32_t hw = __builtin_bit_cast(uint32_t, h);
  const float h0 = __builtin_bit_cast(float, hw << 16);
  const float h1 = __builtin_bit_cast(float, hw & 0xffff0000u);
  const bf16x2 l = __builtin_convertvector(f32x2{r0 - h0, r1 - h1}, bf16x2);
  hi = hw;
  lo = __builtin_bit_cast(uint32_t, l);
}

// SCHED = 0 pins each group (its MFMAs, fragment reads and epilogue pair)
// in program order; SCHED = 1 leaves the order of the tile's instructions to
// the compiler, which may interleave the independent MFMA chains of
// neighbouring groups (a forward and an adjoint group never depend on each
// other).
template <int FAM, int P, int FWD, bool VALUE, int FK, int SCHED>
__global__ __launch_bounds__(512) void k_mfma32(MfmaArgs a) {
  constexpr int KB = P / 16;                 // forward K blocks
  constexpr int MB = P / 32;                 // adjoint M blocks
  constexpr int NFF = m2_nfrag_fwd(P);
  constexpr int NF = m2_nfrag(P);
  constexpr int NST = NF * 64 / (64 * MF_WAVES);  // uint4 staged per thread
  constexpr int NT = FWD == 5 ? 3 : 2;
  constexpr int NBUF = 4;
  constexpr int NG = KB + 2 * MB;            // MFMA groups per tile: forward K blocks, adjoint (M block, K half)
  // LDS fragment reads run PF groups ahead of their MFMAs (two where the
  // registers allow it: the p = 128 kernels need theirs for operands)
  constexpr int PF = P == 64 ? 2 : 1;
  static_assert(NST * 64 * MF_WAVES == NF * 64, "staging must tile the fragments");
  static_assert(NST == 2 || NST == 4, "two or four staged vectors per thread");
  static_assert(NG == 8 || NG == 16, "8 or 16 groups per tile");

  __shared__ __align__(16) uint4 sfrag[NBUF][NF * 64];
  __shared__ __align__(16) float sy[NBUF][MF_ROWS];
  __shared__ __align__(16) int32_t sf[NBUF][MF_ROWS];
  __shared__ uint32_t sflag[NBUF];

  const DevModel& m = a.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int hh = lane >> 5;
  const int l32 = lane & 31;
  const int task = mf_xcd_task(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int n_ct = static_cast<int>((m.C + MF_CHAIN_TILE - 1) / MF_CHAIN_TILE);
  const int sp = task / n_ct;
  const int ct = task - sp * n_ct;
  const int64_t cbase = static_cast<int64_t>(ct) * MF_CHAIN_TILE + wave * MF_CHAINS_PER_WAVE;
  const bool wave_active = cbase < m.C;
  const int t_beg = sp * a.tiles_per_split;
  const int t_end = min(a.n_tiles, t_beg + a.tiles_per_split);
  const int t_last = t_end > t_beg ? t_end - 1 : t_beg;

  // this lane's chain (lanes l and l + 32 share it)
  const int64_t cidx = cbase + l32;
  const bool cvalid = cidx < m.C;
  const int kf = fold_of_chain(m, cvalid ? cidx : m.C - 1);
  int elo = 0, ehi = 0;
  if (FK == PCV_FOLDS_INTERVALS) {
    elo = m.ivals[4 * kf + 2];
    ehi = m.ivals[4 * kf + 3];
  }

  // theta as the B operand: lane holds theta[16 kb + 8 hh + e][chain]
  bf16x8 th[NT][KB];
  if (m.mmask) mf_theta_terms<FAM, NT, KB, 16, true>(m, cidx, 8 * hh, th);
  else mf_theta_terms<FAM, NT, KB, 16, false>(m, cidx, 8 * hh, th);

  f32x16 gacc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int i = 0; i < 16; ++i) gacc[mb][i] = 0.f;
  double vacc = 0.0;
  const float is2 = static_cast<float>(m.inv_sigma2);
  const int nrows = static_cast<int>(m.n);

  // ---- staging: global -> registers -> LDS ring ---------------------------
  uint4 st0, st1, st2, st3;
  float my_y = 0.f;
  int32_t my_f = 0;
  uint32_t my_flag = 0;
  auto load_stage = [&](int tt) {
    const uint4* src = a.Xpk + static_cast<int64_t>(tt) * NF * 64;
    st0 = src[tid];
    st1 = src[512 + tid];
    if constexpr (NST == 4) {
      st2 = src[1024 + tid];
      st3 = src[1536 + tid];
    }
    my_y = a.ty[static_cast<int64_t>(tt) * MF_ROWS + (tid & (MF_ROWS - 1))];
    my_f = a.tfid[static_cast<int64_t>(tt) * MF_ROWS + (tid & (MF_ROWS - 1))];
    my_flag = a.tflag[static_cast<int64_t>(tt) * n_ct + ct];
  };
  auto store_stage = [&](int b) {
    sfrag[b][tid] = st0;
    sfrag[b][512 + tid] = st1;
    if constexpr (NST == 4) {
      sfrag[b][1024 + tid] = st2;
      sfrag[b][1536 + tid] = st3;
    }
    sy[b][tid & (MF_ROWS - 1)] = my_y;
    sf[b][tid & (MF_ROWS - 1)] = my_f;
    if (tid == 0) sflag[b] = my_flag;
  };
  auto frag = [&](int b, int f) { return __builtin_bit_cast(bf16x8, sfrag[b][f * 64 + lane]); };
  // group g: even g -> forward K block g/2 (next tile), odd g -> adjoint (M
  // block, K half) number g/2 (previous tile); both read two fragments
  auto group_frag_index = [&](int g) {
    return (g & 1) ? NFF + (g >> 1) * 2 : (g >> 1) * 2;
  };

  // prologue, as in k_mfma: slot 3 stands in for tile t_beg - 1 (zero residuals)
  load_stage(t_beg < t_last ? t_beg : t_last);
  store_stage(0);
  store_stage(3);
  load_stage(min(t_beg + 1, t_last));
  store_stage(1);
  load_stage(min(t_beg + 2, t_last));
  __syncthreads();
  f32x16 eta_cur, eta_nxt;
#pragma unroll
  for (int i = 0; i < 16; ++i) eta_cur[i] = 0.f;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const bf16x8 x0 = frag(0, 2 * kb), x1 = frag(0, 2 * kb + 1);
    eta_cur = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, th[0][kb], eta_cur, 0, 0, 0);
    eta_cur = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, th[1][kb], eta_cur, 0, 0, 0);
    eta_cur = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, th[0][kb], eta_cur, 0, 0, 0);
    if (NT == 3) {
      eta_cur = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, th[NT - 1][kb], eta_cur, 0, 0, 0);
      eta_cur = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, th[1][kb], eta_cur, 0, 0, 0);
    }
  }
  // residual operands (as packed bf16 words): previous / current tile, K halves
  u32x4 rph[2], rpl[2], rch[2], rcl[2];
#pragma unroll
  for (int kh = 0; kh < 2; ++kh) {
    rph[kh] = u32x4{0u, 0u, 0u, 0u};
    rpl[kh] = u32x4{0u, 0u, 0u, 0u};
    rch[kh] = rph[kh];
    rcl[kh] = rpl[kh];
  }

  for (int tt = t_beg; tt < t_end; ++tt) {
    const int i = tt - t_beg;
    const int bc = i & 3, b1 = (i + 1) & 3, b2 = (i + 2) & 3, bp = (i + 3) & 3;
    __syncthreads();
    store_stage(b2);
    load_stage(min(tt + 3, t_last));
    const uint32_t flag = __builtin_amdgcn_readfirstlane(sflag[bc]);
#pragma unroll
    for (int q = 0; q < 16; ++q) eta_nxt[q] = 0.f;
    float vt = 0.f;

    // the epilogue of tile tt, one pair of elements per slot, spread over
    // the tile's MFMA groups; waves whose flag bit is set apply the fold and
    // row masks (a wave-uniform branch around the mask arithmetic only)
    const bool masked = (flag >> wave) & 1u;
    // y of this lane's 16 rows of the tile: rows 8q + 4hh + (0..3)
    f32x4 yq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) yq[q] = *reinterpret_cast<const f32x4*>(&sy[bc][8 * q + 4 * hh]);
    // fragments of groups g .. g + PF are in flight (ring of PF + 1 groups)
    bf16x8 xr0[PF + 1], xr1[PF + 1];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int bn = (q & 1) ? bp : b1;
      xr0[q] = frag(bn, group_frag_index(q));
      xr1[q] = frag(bn, group_frag_index(q) + 1);
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      if (g + PF < NG) {
        const int bn = ((g + PF) & 1) ? bp : b1;
        xr0[(g + PF) % (PF + 1)] = frag(bn, group_frag_index(g + PF));
        xr1[(g + PF) % (PF + 1)] = frag(bn, group_frag_index(g + PF) + 1);
      }
      const bf16x8 xa0 = xr0[g % (PF + 1)], xa1 = xr1[g % (PF + 1)];
      if ((g & 1) == 0) {
        const int kb = g >> 1;
        f32x16 acc = eta_nxt;
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa0, th[0][kb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa0, th[1][kb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa1, th[0][kb], acc, 0, 0, 0);
        if (NT == 3) {
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa0, th[NT - 1][kb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa1, th[1][kb], acc, 0, 0, 0);
        }
        eta_nxt = acc;
      } else {
        const int mb = (g >> 1) >> 1, kh = (g >> 1) & 1;
        const bf16x8 rh = __builtin_bit_cast(bf16x8, rph[kh]);
        const bf16x8 rl = __builtin_bit_cast(bf16x8, rpl[kh]);
        f32x16 acc = gacc[mb];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa0, rh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa0, rl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa1, rh, acc, 0, 0, 0);
        gacc[mb] = acc;
      }
      // epilogue pairs [g*8/NG, (g+1)*8/NG) of tile tt: elements 2u, 2u+1.
      // Gradient launches compute every residual unmasked here and clear
      // the non-train ones after the loop; value launches mask in place.
#pragma unroll
      for (int u = (g * 8) / NG; u < ((g + 1) * 8) / NG; ++u) {
        const int e0 = 2 * u;
        const int rl0 = m2_row(e0, hh);          // rows rl0, rl0 + 1 of the tile
        float r[2], l0[2] = {0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float yv = yq[e0 >> 2][(e0 & 3) + q];
          if (VALUE) mf_resid_ell0<FAM>(yv, eta_cur[e0 + q], is2, r[q], l0[q]);
          else r[q] = mf_resid<FAM>(yv, eta_cur[e0 + q], is2);
          if (VALUE) {
            const int row = tt * MF_ROWS + rl0 + q;
            bool train = row < nrows;
            if (FK == PCV_FOLDS_INDEX) train = train & (sf[bc][rl0 + q] != kf);
            else train = train & ((row < elo) | (row >= ehi));
            r[q] = train ? r[q] : 0.f;
            vt += train ? l0[q] : 0.f;
          }
        }
        uint32_t hw, lw;
        m2_split2(r[0], r[1], hw, lw);
        const int kh = e0 >> 3, w = (e0 & 7) >> 1;
        rch[kh][w] = hw;
        rcl[kh][w] = lw;
      }
      if constexpr (SCHED == 0) __builtin_amdgcn_sched_barrier(0);
    }
    if (!VALUE && masked) {
      // this wave's chains have non-train (or padded) rows in the tile:
      // clear their residuals (both bf16 terms) before the adjoint uses them
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int rl = m2_row(e, hh);
        const int row = tt * MF_ROWS + rl;
        bool train = row < nrows;
        if (FK == PCV_FOLDS_INDEX) train = train & (sf[bc][rl] != kf);
        else train = train & ((row < elo) | (row >= ehi));
        const uint32_t keep = train ? 0xFFFFFFFFu : ((e & 1) ? 0x0000FFFFu : 0xFFFF0000u);
        const int kh = e >> 3, w = (e & 7) >> 1;
        rch[kh][w] &= keep;
        rcl[kh][w] &= keep;
      }
    }

    if (VALUE) vacc += static_cast<double>(vt);
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      rph[kh] = rch[kh];
      rpl[kh] = rcl[kh];
    }
    eta_cur = eta_nxt;
  }
  // adjoint of the last tile
  {
    const int bl = (t_end - 1 - t_beg) & 3;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int kh = 0; kh < 2; ++kh) {
        const int f = NFF + (mb * 2 + kh) * 2;
        const bf16x8 x0 = frag(bl, f), x1 = frag(bl, f + 1);
        const bf16x8 rh = __builtin_bit_cast(bf16x8, rph[kh]);
        const bf16x8 rl = __builtin_bit_cast(bf16x8, rpl[kh]);
        f32x16 acc = gacc[mb];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, rh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, rl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, rh, acc, 0, 0, 0);
        gacc[mb] = acc;
      }
    }
  }

  if (!wave_active) return;
  if (cvalid) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int j = mb * 32 + m2_row(q, hh);
        if (j < m.p) a.Gpart[(static_cast<int64_t>(sp) * m.p + j) * m.C + cidx] = gacc[mb][q];
      }
  }
  if (VALUE) {
    double v = vacc;
    v += __shfl_xor(v, 32);
    if (lane < 32 && cvalid) a.Vpart[static_cast<int64_t>(sp) * m.C + cidx] = v * mf_ell0_scale<FAM>();
  }
}

// Pack X (fp64, row-major, p columns) for k_mfma32 at width P >= p (zero
// columns past p), split hi/lo: forward fragment
// (kb, plane) lane l holds row l%32, columns 16 kb + 8 (l/32) + e; adjoint
// fragment (mb, kh, plane) lane l holds column 32 mb + l%32 at the rows of
// K half kh in accumulator order (m2_row).
__global__ void k_mfma32_pack(const double* __restrict__ X, int64_t n, int p, int P, int n_tiles,
                              uint4* __restrict__ out) {
  const int nf = m2_nfrag(P), nff = m2_nfrag_fwd(P);
  const int64_t total = static_cast<int64_t>(n_tiles) * nf * 64;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int lane = static_cast<int>(idx % 64);
    const int f = static_cast<int>((idx / 64) % nf);
    const int64_t tt = idx / (64 * nf);
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t row0 = tt * MF_ROWS;
    const int plane = f & 1;
    bf16x8 v;
    if (f < nff) {
      const int kb = f >> 1;
      const int64_t row = row0 + l32;
      for (int e = 0; e < 8; ++e) {
        const int col = kb * 16 + 8 * h + e;
        const float x = row < n && col < p ? static_cast<float>(X[row * p + col]) : 0.f;
        const __bf16 hb = to_bf16(x);
        v[e] = plane == 0 ? hb : to_bf16(x - static_cast<float>(hb));
      }
    } else {
      const int blk = (f - nff) >> 1;        // mb * 2 + kh
      const int mb = blk >> 1, kh = blk & 1;
      const int col = mb * 32 + l32;
      for (int e = 0; e < 8; ++e) {
        const int64_t row = row0 + 16 * kh + m2_row(e, h);
        const float x = row < n && col < p ? static_cast<float>(X[row * p + col]) : 0.f;
        const __bf16 hb = to_bf16(x);
        v[e] = plane == 0 ? hb : to_bf16(x - static_cast<float>(hb));
      }
    }
    out[idx] = __builtin_bit_cast(uint4, v);
  }
}

// Pack X (fp64, row-major, p columns) into the two fragment orders at width
// P >= p (zero columns past p), split hi/lo.
__global__ void k_mfma_pack(const double* __restrict__ X, int64_t n, int p, int P, int n_tiles,
                            uint4* __restrict__ out) {
  const int nf = mf_nfrag(P), nff = mf_nfrag_fwd(P), KB = P / 32;
  const int64_t total = static_cast<int64_t>(n_tiles) * nf * 64;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int lane = static_cast<int>(idx % 64);
    const int f = static_cast<int>((idx / 64) % nf);
    const int64_t tt = idx / (64 * nf);
    const int g4 = lane >> 4, l16 = lane & 15;
    const int64_t row0 = tt * MF_ROWS;
    bf16x8 v;
    int plane;
    if (f < nff) {
      plane = f & 1;
      const int kb = (f >> 1) % KB, mh = (f >> 1) / KB;
      const int64_t row = row0 + mh * 16 + l16;
      for (int e = 0; e < 8; ++e) {
        const int col = kb * 32 + 8 * g4 + e;
        const float x = row < n && col < p ? static_cast<float>(X[row * p + col]) : 0.f;
        const __bf16 h = to_bf16(x);
        v[e] = plane == 0 ? h : to_bf16(x - static_cast<float>(h));
      }
    } else {
      const int ff = f - nff;
      plane = ff & 1;
      const int mb = ff >> 1;
      const int col = mb * 16 + l16;
      for (int e = 0; e < 8; ++e) {
        const int64_t row = row0 + (e < 4 ? 4 * g4 + e : 16 + 4 * g4 + (e - 4));
        const float x = row < n && col < p ? static_cast<float>(X[row * p + col]) : 0.f;
        const __bf16 h = to_bf16(x);
        v[e] = plane == 0 ? h : to_bf16(x - static_cast<float>(h));
      }
    }
    out[idx] = __builtin_bit_cast(uint4, v);
  }
}

template <int FAM, int P, int FWD, int SHAPE>
static hipError_t launch_mfma_p(const MfmaArgs& a, bool value, int nblk, hipStream_t st) {
  const bool iv = a.m.fold_kind == PCV_FOLDS_INTERVALS;
#define PCV_MFMA_LAUNCH(KERN, ...)                                                                         \
  do {                                                                                                   \
    if (value) {                                                                                         \
      if (iv) hipLaunchKernelGGL((KERN<FAM, P, FWD, true, PCV_FOLDS_INTERVALS __VA_ARGS__>), dim3(nblk), dim3(512), 0, st, a); \
      else hipLaunchKernelGGL((KERN<FAM, P, FWD, true, PCV_FOLDS_INDEX __VA_ARGS__>), dim3(nblk), dim3(512), 0, st, a);       \
    } else {                                                                                             \
      if (iv) hipLaunchKernelGGL((KERN<FAM, P, FWD, false, PCV_FOLDS_INTERVALS __VA_ARGS__>), dim3(nblk), dim3(512), 0, st, a); \
      else hipLaunchKernelGGL((KERN<FAM, P, FWD, false, PCV_FOLDS_INDEX __VA_ARGS__>), dim3(nblk), dim3(512), 0, st, a);       \
    }                                                                                                    \
  } while (0)
  if constexpr (SHAPE == MFMA_SHAPE_32X32X16) PCV_MFMA_LAUNCH(k_mfma32, , 0);
  else if constexpr (SHAPE == MFMA_SHAPE_32X32X16_IL) PCV_MFMA_LAUNCH(k_mfma32, , 1);
  else if constexpr (SHAPE == MFMA_SHAPE_16X16X32_C16) {
    if constexpr (P == 64) PCV_MFMA_LAUNCH(k_mfma, , 1);
    else return hipErrorInvalidValue;
  } else PCV_MFMA_LAUNCH(k_mfma, , 2);
#undef PCV_MFMA_LAUNCH
  return hipGetLastError();
}

template <int FAM, int SHAPE>
static hipError_t launch_mfma_f(const MfmaArgs& a, int P, int fwd, bool value, int nblk, hipStream_t st) {
  if (P == 64 && fwd == 3) return launch_mfma_p<FAM, 64, 3, SHAPE>(a, value, nblk, st);
  if (P == 64 && fwd == 5) return launch_mfma_p<FAM, 64, 5, SHAPE>(a, value, nblk, st);
  if (P == 128 && fwd == 3) return launch_mfma_p<FAM, 128, 3, SHAPE>(a, value, nblk, st);
  if (P == 128 && fwd == 5) return launch_mfma_p<FAM, 128, 5, SHAPE>(a, value, nblk, st);
  return hipErrorInvalidValue;
}

template <int SHAPE>
static hipError_t launch_mfma_s(const MfmaArgs& a, int P, int fwd, bool value, int nblk, hipStream_t st) {
  switch (a.m.family) {
    case FAM_GAUSS: return launch_mfma_f<FAM_GAUSS, SHAPE>(a, P, fwd, value, nblk, st);
    case FAM_LOGIT: return launch_mfma_f<FAM_LOGIT, SHAPE>(a, P, fwd, value, nblk, st);
    case FAM_POIS: return launch_mfma_f<FAM_POIS, SHAPE>(a, P, fwd, value, nblk, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mfma(const DevModel& m, int shape, const uint4* Xpk, const float* ty, const int32_t* tfid,
                       const uint32_t* tflag, float* Gpart, double* Vpart, int n_tiles, int tiles_per_split,
                       int n_splits, int fwd, bool value, hipStream_t st) {
  MfmaArgs a;
  a.m = m;
  a.Xpk = Xpk;
  a.ty = ty;
  a.tfid = tfid;
  a.tflag = tflag;
  a.Gpart = Gpart;
  a.Vpart = Vpart;
  a.n_tiles = n_tiles;
  a.tiles_per_split = tiles_per_split;
  a.n_splits = n_splits;
  const int ct = mfma_chain_tile(shape);
  const int n_ct = static_cast<int>((m.C + ct - 1) / ct);
  const int nblk = n_ct * n_splits;
  const int P = mfma_width(m.p);
  if (shape == MFMA_SHAPE_32X32X16) return launch_mfma_s<MFMA_SHAPE_32X32X16>(a, P, fwd, value, nblk, st);
  if (shape == MFMA_SHAPE_32X32X16_IL) return launch_mfma_s<MFMA_SHAPE_32X32X16_IL>(a, P, fwd, value, nblk, st);
  if (shape == MFMA_SHAPE_16X16X32) return launch_mfma_s<MFMA_SHAPE_16X16X32>(a, P, fwd, value, nblk, st);
  if (shape == MFMA_SHAPE_16X16X32_C16 && P == 64)
    return launch_mfma_s<MFMA_SHAPE_16X16X32_C16>(a, P, fwd, value, nblk, st);
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_pack(const double* X, int64_t n, int p, int n_tiles, int shape, uint4* out, hipStream_t st) {
  const int P = mfma_width(p);
  if (mfma_layout(shape) == 1)
    hipLaunchKernelGGL(k_mfma32_pack, dim3(1024), dim3(256), 0, st, X, n, p, P, n_tiles, out);
  else hipLaunchKernelGGL(k_mfma_pack, dim3(1024), dim3(256), 0, st, X, n, p, P, n_tiles, out);
  return hipGetLastError();
}

int mfma_chain_tile(int shape) { return shape == MFMA_SHAPE_16X16X32_C16 ? MF_CHAIN_TILE / 2 : MF_CHAIN_TILE; }
int mfma_rows_per_tile() { return MF_ROWS; }
// X packing of a shape: 0 = the 16x16x32 kernels' fragment orders, 1 = the 32x32x16 kernels'
int mfma_layout(int shape) { return shape == MFMA_SHAPE_32X32X16 || shape == MFMA_SHAPE_32X32X16_IL ? 1 : 0; }
bool mfma_shape_ok(int shape, int64_t p) {
  return shape >= MFMA_SHAPE_16X16X32 && shape <= MFMA_SHAPE_16X16X32_C16 &&
         (shape != MFMA_SHAPE_16X16X32_C16 || mfma_width(p) == 64);
}
int mfma_nfrag(int p, int shape) {
  const int P = mfma_width(p);
  return mfma_layout(shape) == 1 ? m2_nfrag(P) : mf_nfrag(P);
}

}  // namespace pcv
