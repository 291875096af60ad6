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
  int n_tiles, tiles_per_split, n_splits;
};

__device__ __forceinline__ __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }

template <int FAM, int P, int FWD, bool VALUE>
__global__ __launch_bounds__(512) void k_mfma(MfmaArgs a) {
  constexpr int KB = P / 32;
  constexpr int MB = P / 16;
  constexpr int NFF = mf_nfrag_fwd(P);
  constexpr int NF = mf_nfrag(P);
  constexpr int NST = NF * 64 / (64 * MF_WAVES);  // uint4 staged per thread
  constexpr int NT = FWD == 5 ? 3 : 2;             // theta terms
  static_assert(NST * 64 * MF_WAVES == NF * 64, "staging must tile the fragments");

  __shared__ __align__(16) uint4 sfrag[NF * 64];
  __shared__ float sy[MF_ROWS];
  __shared__ int32_t sf[MF_ROWS];

  const DevModel& m = a.m;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g4 = lane >> 4;
  const int l16 = lane & 15;
  const int ct = blockIdx.x / a.n_splits;
  const int sp = blockIdx.x - ct * a.n_splits;
  const int64_t cbase = static_cast<int64_t>(ct) * MF_CHAIN_TILE + wave * MF_CHAINS_PER_WAVE;
  const bool wave_active = cbase < m.C;
  const int t_beg = sp * a.tiles_per_split;
  const int t_end = min(a.n_tiles, t_beg + a.tiles_per_split);

  // chains of this lane in its two 16-chain blocks
  int kf[2], elo[2], ehi[2];
  int64_t cidx[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int64_t c = cbase + cb * 16 + l16;
    cidx[cb] = c;
    const int64_t cc = c < m.C ? c : m.C - 1;
    kf[cb] = static_cast<int>(cc / m.L);
    elo[cb] = 0;
    ehi[cb] = 0;
    if (m.fold_kind == PCV_FOLDS_INTERVALS) {
      elo[cb] = m.ivals[4 * kf[cb] + 2];
      ehi[cb] = m.ivals[4 * kf[cb] + 3];
    }
  }

  // theta operand fragments: lane holds theta[k = kb*32 + 8*g4 + e][chain]
  bf16x8 th[NT][KB][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int64_t c = cidx[cb];
    const bool cv = c < m.C;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = kb * 32 + 8 * g4 + e;
        const double t = cv ? m.q1[static_cast<int64_t>(j) * m.C + c] : 0.0;
        if (NT == 2) {
          const float t32 = static_cast<float>(t);
          const __bf16 h = to_bf16(t32);
          th[0][kb][cb][e] = h;
          th[1][kb][cb][e] = to_bf16(t32 - static_cast<float>(h));
        } else {
          const __bf16 h = to_bf16(static_cast<float>(t));
          const double r1 = t - static_cast<double>(static_cast<float>(h));
          const __bf16 mdl = to_bf16(static_cast<float>(r1));
          const double r2 = r1 - static_cast<double>(static_cast<float>(mdl));
          th[0][kb][cb][e] = h;
          th[1][kb][cb][e] = mdl;
          th[NT - 1][kb][cb][e] = to_bf16(static_cast<float>(r2));
        }
      }
    }
  }

  f32x4 gacc[MB][2];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) gacc[mb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  double vacc[2] = {0.0, 0.0};
  const float is2 = static_cast<float>(m.inv_sigma2);

  // register staging of the next tile (the clamped index keeps the last,
  // redundant prefetch inside the buffer)
  static_assert(NST == 2 || NST == 4, "two or four staged vectors per thread");
  uint4 st0, st1, st2, st3;   // named registers: a private array here ends up in scratch
  float my_y = 0.f;
  int32_t my_f = 0;
  const int t_last = t_end > t_beg ? t_end - 1 : t_beg;
  {
    const int tt0 = min(t_beg, a.n_tiles - 1);
    const uint4* src = a.Xpk + static_cast<int64_t>(tt0) * NF * 64;
    st0 = src[tid];
    st1 = src[512 + tid];
    if constexpr (NST == 4) {
      st2 = src[1024 + tid];
      st3 = src[1536 + tid];
    }
    if (tid < MF_ROWS) {
      my_y = a.ty[static_cast<int64_t>(tt0) * MF_ROWS + tid];
      my_f = a.tfid[static_cast<int64_t>(tt0) * MF_ROWS + tid];
    }
  }

  for (int tt = t_beg; tt < t_end; ++tt) {
    __syncthreads();
    sfrag[tid] = st0;
    sfrag[512 + tid] = st1;
    if constexpr (NST == 4) {
      sfrag[1024 + tid] = st2;
      sfrag[1536 + tid] = st3;
    }
    if (tid < MF_ROWS) {
      sy[tid] = my_y;
      sf[tid] = my_f;
    }
    __syncthreads();
    {
      const int tn = min(tt + 1, t_last);
      const uint4* src = a.Xpk + static_cast<int64_t>(tn) * NF * 64;
      st0 = src[tid];
      st1 = src[512 + tid];
      if constexpr (NST == 4) {
        st2 = src[1024 + tid];
        st3 = src[1536 + tid];
      }
      if (tid < MF_ROWS) {
        my_y = a.ty[static_cast<int64_t>(tn) * MF_ROWS + tid];
        my_f = a.tfid[static_cast<int64_t>(tn) * MF_ROWS + tid];
      }
    }
    if (!wave_active) continue;

    // ---- forward: eta[32 rows x 32 chains] -------------------------------
    f32x4 eta[2][2];
#pragma unroll
    for (int mh = 0; mh < 2; ++mh)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) eta[mh][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int mh = 0; mh < 2; ++mh) {
        const int f = (mh * KB + kb) * 2;
        const bf16x8 x0 = __builtin_bit_cast(bf16x8, sfrag[f * 64 + lane]);
        const bf16x8 x1 = __builtin_bit_cast(bf16x8, sfrag[(f + 1) * 64 + lane]);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
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

    // ---- epilogue: masked residual, split into bf16 hi/lo ----------------
    bf16x8 rhi[2], rlo[2];
#pragma unroll
    for (int mh = 0; mh < 2; ++mh) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rl = mh * 16 + 4 * g4 + i;
        const int64_t row = static_cast<int64_t>(tt) * MF_ROWS + rl;
        const float y = sy[rl];
        const int fr = sf[rl];
        const bool rv = row < m.n;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          bool train;
          if (m.fold_kind == PCV_FOLDS_INDEX) train = rv && (fr != kf[cb]);
          else if (m.fold_kind == PCV_FOLDS_INTERVALS) train = rv && ((row < elo[cb]) || (row >= ehi[cb]));
          else train = rv && (m.roles[static_cast<int64_t>(kf[cb]) * m.n + row] == 1);
          const float e = eta[mh][cb][i];
          const float r = train ? resid32<FAM>(y, e, is2) : 0.f;
          if (VALUE) {
            if (train) vacc[cb] += static_cast<double>(ell0_32<FAM>(y, e, is2));
          }
          const __bf16 h = to_bf16(r);
          rhi[cb][mh * 4 + i] = h;
          rlo[cb][mh * 4 + i] = to_bf16(r - static_cast<float>(h));
        }
      }
    }

    // ---- adjoint: G[P x 32 chains] += X' R ------------------------------
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int f = NFF + mb * 2;
      const bf16x8 x0 = __builtin_bit_cast(bf16x8, sfrag[f * 64 + lane]);
      const bf16x8 x1 = __builtin_bit_cast(bf16x8, sfrag[(f + 1) * 64 + lane]);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        f32x4 acc = gacc[mb][cb];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, rhi[cb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, rlo[cb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, rhi[cb], acc, 0, 0, 0);
        gacc[mb][cb] = acc;
      }
    }
  }

  if (!wave_active) return;
  // ---- partial results -----------------------------------------------------
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int64_t c = cidx[cb];
    if (c < m.C) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = mb * 16 + 4 * g4 + i;
          a.Gpart[(static_cast<int64_t>(sp) * P + j) * m.C + c] = gacc[mb][cb][i];
        }
    }
    if (VALUE) {
      double v = vacc[cb];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16 && c < m.C) a.Vpart[static_cast<int64_t>(sp) * m.C + c] = v;
    }
  }
}

// Pack X (fp64, row-major) into the two fragment orders, split hi/lo.
__global__ void k_mfma_pack(const double* __restrict__ X, int64_t n, int P, int n_tiles, uint4* __restrict__ out) {
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
        const float x = row < n ? static_cast<float>(X[row * P + col]) : 0.f;
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
        const float x = row < n ? static_cast<float>(X[row * P + col]) : 0.f;
        const __bf16 h = to_bf16(x);
        v[e] = plane == 0 ? h : to_bf16(x - static_cast<float>(h));
      }
    }
    out[idx] = __builtin_bit_cast(uint4, v);
  }
}

template <int FAM, int P, int FWD>
static hipError_t launch_mfma_p(const MfmaArgs& a, bool value, int nblk, hipStream_t st) {
  if (value) hipLaunchKernelGGL((k_mfma<FAM, P, FWD, true>), dim3(nblk), dim3(512), 0, st, a);
  else hipLaunchKernelGGL((k_mfma<FAM, P, FWD, false>), dim3(nblk), dim3(512), 0, st, a);
  return hipGetLastError();
}

template <int FAM>
static hipError_t launch_mfma_f(const MfmaArgs& a, int P, int fwd, bool value, int nblk, hipStream_t st) {
  if (P == 64 && fwd == 3) return launch_mfma_p<FAM, 64, 3>(a, value, nblk, st);
  if (P == 64 && fwd == 5) return launch_mfma_p<FAM, 64, 5>(a, value, nblk, st);
  if (P == 128 && fwd == 3) return launch_mfma_p<FAM, 128, 3>(a, value, nblk, st);
  if (P == 128 && fwd == 5) return launch_mfma_p<FAM, 128, 5>(a, value, nblk, st);
  return hipErrorInvalidValue;
}

hipError_t launch_mfma(const DevModel& m, const uint4* Xpk, const float* ty, const int32_t* tfid, float* Gpart,
                       double* Vpart, int n_tiles, int tiles_per_split, int n_splits, int fwd, bool value,
                       hipStream_t st) {
  MfmaArgs a;
  a.m = m;
  a.Xpk = Xpk;
  a.ty = ty;
  a.tfid = tfid;
  a.Gpart = Gpart;
  a.Vpart = Vpart;
  a.n_tiles = n_tiles;
  a.tiles_per_split = tiles_per_split;
  a.n_splits = n_splits;
  const int n_ct = static_cast<int>((m.C + MF_CHAIN_TILE - 1) / MF_CHAIN_TILE);
  const int nblk = n_ct * n_splits;
  const int P = static_cast<int>(m.p);
  switch (m.family) {
    case FAM_GAUSS: return launch_mfma_f<FAM_GAUSS>(a, P, fwd, value, nblk, st);
    case FAM_LOGIT: return launch_mfma_f<FAM_LOGIT>(a, P, fwd, value, nblk, st);
    case FAM_POIS: return launch_mfma_f<FAM_POIS>(a, P, fwd, value, nblk, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_pack(const double* X, int64_t n, int P, int n_tiles, uint4* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mfma_pack, dim3(1024), dim3(256), 0, st, X, n, P, n_tiles, out);
  return hipGetLastError();
}

int mfma_chain_tile() { return MF_CHAIN_TILE; }
int mfma_rows_per_tile() { return MF_ROWS; }
int mfma_nfrag(int P) { return mf_nfrag(P); }

}  // namespace pcv
