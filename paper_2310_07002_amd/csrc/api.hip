// Host runtime of the PCV library: validation, device buffers, path
// selection, transition scheduling and the C ABI declared in include/pcv.h.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pcv_internal.h"

namespace pcv {
// launchers (k_valu.hip, k_mfma.hip, k_common.hip)
hipError_t launch_valu(const DevModel& m, const void* Xv, bool fp64, int pb, int W, int mode, int64_t t0,
                       int n_iter, int n_steps, hipStream_t st);
size_t valu_smem_bytes(bool fp64, int W, int family, int n_groups, int pb);
int valu_part_occupancy(bool fp64, int family, int pb, int W, size_t smem);
hipError_t launch_valu_part(const DevModel& m, const void* Xv, bool fp64, int pb, int W, int ns, double* Gpart,
                            double* Vpart, double* uscr, bool value, bool series, hipStream_t st);
hipError_t launch_valu_finish(const DevModel& m, const double* Gpart, const double* uscr, int ns, int mode,
                              hipStream_t st);
int valu_pb(int64_t p, bool fp64);
hipError_t launch_mfma(const DevModel& m, int shape, const uint4* Xpk, const float* ty, const int32_t* tfid,
                       const uint32_t* tflag, float* Gpart, double* Vpart, int n_tiles, int tiles_per_split,
                       int n_splits, int fwd, bool value, hipStream_t st);
hipError_t launch_mfma_pack(const double* X, int64_t n, int p, int n_tiles, int shape, uint4* out, hipStream_t st);
int mfma_chain_tile(int shape);
int mfma_layout(int shape);
bool mfma_shape_ok(int shape, int64_t p);
int mfma_rows_per_tile();
int mfma_nfrag(int p, int shape);
int mfma_width(int64_t p);
hipError_t launch_momentum(const DevModel& m, int64_t t, hipStream_t st);
hipError_t launch_reduce_f32(const DevModel& m, const float* G, int ns, int mode, hipStream_t st);
hipError_t launch_reduce_f64(const DevModel& m, const double* G, int ns, int mode, hipStream_t st);
hipError_t launch_value_finish(const DevModel& m, const double* V, int ns, hipStream_t st);
hipError_t launch_center(const DevModel& m, hipStream_t st);
hipError_t launch_accept(const DevModel& m, const double* V, int ns, int64_t t, hipStream_t st);
hipError_t launch_testlp(const DevModel& m, int max_test_rows, hipStream_t st);
int testlp_groups(int max_test_rows);
hipError_t launch_logpred(const DevModel& m, hipStream_t st);
hipError_t launch_unfused_resid(const DevModel& m, double* eta, int64_t c0, int64_t cc, double* V, int want_value,
                                hipStream_t st);
hipError_t launch_rowconst(const DevModel& m, double* rowc, hipStream_t st);
hipError_t launch_foldconst(const DevModel& m, double prior_const, double* fc, hipStream_t st);
hipError_t launch_to_dc(const double* src, double* dst, int64_t C, int64_t d, hipStream_t st);
hipError_t launch_to_cd(const double* src, double* dst, int64_t C, int64_t d, hipStream_t st);
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t st);
hipError_t launch_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                         uint32_t* out, hipStream_t st);
hipError_t launch_diag(const DevModel& m, int64_t N, double* fold_buf, double* out, hipStream_t st);
hipError_t launch_shuffle(const DevModel& m, int64_t N, int R, uint32_t s0, uint32_t s1, double* rep,
                          double* repmax, hipStream_t st);
hipError_t launch_kick_drift(const DevModel& m, hipStream_t st);
hipError_t launch_tick(const DevModel& m, hipStream_t st);
}  // namespace pcv

using namespace pcv;

enum Path { PATH_VALU = 0, PATH_MFMA = 1, PATH_UNFUSED = 2, PATH_VALU_SPLIT = 3 };

struct pcv_ctx_s {
  DevModel m{};
  int prec = 0, path = 0;
  bool fp64 = true;
  int pb = 0, W = 1;
  bool series = false;   // X is the lag matrix of y (row-split VALU path)
  hipStream_t st = nullptr;
  int64_t t = 0;
  std::vector<void*> allocs;
  // VALU
  void* Xv = nullptr;
  int32_t* wave_rows = nullptr;
  // MFMA
  uint4* Xpk = nullptr;            // X packed for the current MFMA shape
  uint4* Xpk_shape[2] = {nullptr, nullptr};   // packed X per fragment layout (made on first use)
  int mshape = MFMA_SHAPE_32X32X16;
  uint32_t* tflag = nullptr;       // [n_tiles][chain tiles] waves with a non-train or padded row
  float* ty = nullptr;
  int32_t* tfid = nullptr;
  float* Gpart = nullptr;
  double* Vpart = nullptr;
  int n_tiles = 0, tiles_per_split = 0, n_splits = 1, fwd = 3;
  // unfused
  rocblas_handle rb = nullptr;
  double* eta = nullptr;
  double* Gpart64 = nullptr;
  double* theta_cd = nullptr;   // [C][p] copy of theta (chain-major) for the library GEMM
  int unf_splits = 1;           // row splits of the adjoint GEMM (a batched call; k_reduce adds them)
  int64_t unf_rows = 0;         // rows per split (the last split may be shorter)
  int64_t chunk = 0;
  // diagnostics
  double* fold_buf = nullptr;
  double* dscal = nullptr;
  double prior_const = 0.0;
  // captured transition (split paths)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graphs = true;
  int64_t t_host = 0;   // staging for the device counter upload
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double ms_acc = 0.0;
  int64_t n_launch = 0;
  std::string err;
  bool dead = false;
  uint64_t fingerprint = 0;   // of X, y, folds and groups (checkpoints)
  uint64_t fold_fp = 0;       // of the fold set alone (model comparison)
  int split_cap = 0;                    // row splits the partial buffers hold
  int max_test_rows = 0;                // test rows of the largest fold (k_testlp's grid)
  size_t wave_rows_cap = 0;             // row-split VALU: entries the wave_rows buffer holds
  double* uscr = nullptr;               // row-split VALU, hierarchical: [C] log tau of the partials
  std::vector<int32_t> group_of_host;   // row-split VALU, hierarchical: groups of the rows
  std::vector<int32_t> test_ptr_host;   // [K+1] test rows of each fold (CSR)
  std::vector<int64_t> sq_ptr_host;     // [K+1] prefix sums of squared test-set sizes
  double* noalloc_scratch = nullptr;    // this device's copy of the static scratch array
};

namespace {

const char* kGradKernelName[4] = {"k_valu (fused transition)", "k_mfma (bf16 split MFMA value+gradient)",
                                  "rocblas_dgemm + k_unfused_resid (fp64 unfused)", "k_valu_part (row-split VALU value+gradient)"};

// Fingerprint of input arrays (FNV-1a over 8-byte words plus a shift to
// spread high bits; not cryptographic): a checkpoint only resumes a run on
// the same data.
uint64_t fp_mix(uint64_t h, const void* data, size_t bytes) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  size_t i = 0;
  for (; i + 8 <= bytes; i += 8) {
    uint64_t w;
    std::memcpy(&w, b + i, 8);
    h ^= w;
    h *= 0x100000001b3ULL;
    h ^= h >> 29;
  }
  for (; i < bytes; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}

pcv_status fail(pcv_ctx ctx, pcv_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

#define CK(call)                                                                                   \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      ctx->dead = true;                                                                            \
      return fail(ctx, PCV_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));        \
    }                                                                                              \
  } while (0)

template <typename T>
pcv_status dalloc(pcv_ctx ctx, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, PCV_ERR_NOMEM, "hipMalloc failed");
  }
  ctx->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return PCV_OK;
}

#define TRY(x)                       \
  do {                               \
    pcv_status s_ = (x);             \
    if (s_ != PCV_OK) return s_;     \
  } while (0)

template <typename T>
pcv_status upload(pcv_ctx ctx, T** dst, const T* src, size_t count) {
  TRY(dalloc(ctx, dst, count));
  CK(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return PCV_OK;
}

bool usable(pcv_ctx ctx) { return ctx && !ctx->dead; }

void timing_begin(pcv_ctx ctx) {
  if (!ctx->timing) return;
  while (ctx->ev_pool.size() < ctx->ev_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    ctx->ev_pool.push_back(e);
  }
  (void)hipEventRecord(ctx->ev_pool[ctx->ev_used], ctx->st);
}
void timing_end(pcv_ctx ctx) {
  if (!ctx->timing || ctx->ev_pool.size() < ctx->ev_used + 2) return;
  (void)hipEventRecord(ctx->ev_pool[ctx->ev_used + 1], ctx->st);
  ctx->ev_used += 2;
  ctx->n_launch += 1;
}
void timing_collect(pcv_ctx ctx) {
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.f;
    (void)hipEventSynchronize(ctx->ev_pool[i + 1]);
    if (hipEventElapsedTime(&ms, ctx->ev_pool[i], ctx->ev_pool[i + 1]) == hipSuccess) ctx->ms_acc += ms;
  }
  ctx->ev_used = 0;
}

// Partial gradient (and value) at q1 for the split paths.
pcv_status split_partials(pcv_ctx ctx, bool value) {
  DevModel& m = ctx->m;
  if (ctx->path == PATH_VALU_SPLIT) {
    if (ctx->ev_used + 2 > 4096) timing_collect(ctx);
    timing_begin(ctx);
    CK(launch_valu_part(m, ctx->Xv, ctx->fp64, ctx->pb, ctx->W, ctx->n_splits, ctx->Gpart64, ctx->Vpart, ctx->uscr,
                        value, ctx->series, ctx->st));
    timing_end(ctx);
    return PCV_OK;
  }
  if (ctx->path == PATH_MFMA) {
    if (ctx->ev_used + 2 > 4096) timing_collect(ctx);
    timing_begin(ctx);
    CK(launch_mfma(m, ctx->mshape, ctx->Xpk, ctx->ty, ctx->tfid, ctx->tflag, ctx->Gpart, ctx->Vpart, ctx->n_tiles,
                   ctx->tiles_per_split, ctx->n_splits, ctx->fwd, value, ctx->st));
    timing_end(ctx);
    return PCV_OK;
  }
  // unfused fp64: eta = X Theta (library GEMM), residual, G' = R' X (library GEMM).
  // In rocBLAS's column-major terms X [n][p] is p x n and a chain-major copy
  // of theta [C][p] is p x C, so eta (n x chunk, one column per chain) is
  // X^T theta_chunk; G' (chunk x p, written straight into the [p][C]
  // partials) is eta^T X^T.  Of the operand layouts measured for these
  // shapes (small p, long n), these two ran fastest.
  if (ctx->ev_used + 2 > 4096) timing_collect(ctx);
  timing_begin(ctx);
  const double one = 1.0, zero = 0.0;
  CK(launch_to_cd(m.q1, ctx->theta_cd, m.C, m.p, ctx->st));
  for (int64_t c0 = 0; c0 < m.C; c0 += ctx->chunk) {
    const int64_t cc = std::min<int64_t>(ctx->chunk, m.C - c0);
    if (rocblas_dgemm(ctx->rb, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)m.n,
                      (rocblas_int)cc, (rocblas_int)m.p, &one, m.X64, (rocblas_int)m.p, ctx->theta_cd + c0 * m.p,
                      (rocblas_int)m.p, &zero, ctx->eta, (rocblas_int)m.n) != rocblas_status_success)
      return fail(ctx, PCV_ERR_DEVICE, "rocblas_dgemm (eta) failed");
    CK(launch_unfused_resid(m, ctx->eta, c0, cc, ctx->Vpart, value ? 1 : 0, ctx->st));
    // the adjoint's output is only chunk x p, so its rows are split into
    // independent products of one batched call (enough tiles to fill the
    // chip); the partials are summed in split order by k_reduce
    const int64_t rs = ctx->unf_rows;
    const int64_t full = m.n / rs, rem = m.n - full * rs;
    if (full > 0 &&
        rocblas_dgemm_strided_batched(ctx->rb, rocblas_operation_transpose, rocblas_operation_transpose,
                                      (rocblas_int)cc, (rocblas_int)m.p, (rocblas_int)rs, &one, ctx->eta,
                                      (rocblas_int)m.n, (rocblas_stride)rs, m.X64, (rocblas_int)m.p,
                                      (rocblas_stride)(rs * m.p), &zero, ctx->Gpart64 + c0, (rocblas_int)m.C,
                                      (rocblas_stride)(m.p * m.C), (rocblas_int)full) != rocblas_status_success)
      return fail(ctx, PCV_ERR_DEVICE, "rocblas_dgemm_strided_batched (gradient) failed");
    if (rem > 0 &&
        rocblas_dgemm(ctx->rb, rocblas_operation_transpose, rocblas_operation_transpose, (rocblas_int)cc,
                      (rocblas_int)m.p, (rocblas_int)rem, &one, ctx->eta + full * rs, (rocblas_int)m.n,
                      m.X64 + full * rs * m.p, (rocblas_int)m.p, &zero, ctx->Gpart64 + full * m.p * m.C + c0,
                      (rocblas_int)m.C) != rocblas_status_success)
      return fail(ctx, PCV_ERR_DEVICE, "rocblas_dgemm (gradient) failed");
  }
  timing_end(ctx);
  return PCV_OK;
}

pcv_status split_reduce(pcv_ctx ctx, int mode) {
  if (ctx->path == PATH_VALU_SPLIT) {
    // the split sums, prior (and hierarchical chain rule) and update per
    // (entry, chain) thread
    if (hier_family(ctx->m.family)) {
      CK(launch_valu_finish(ctx->m, ctx->Gpart64, ctx->uscr, ctx->n_splits, mode, ctx->st));
    } else {
      CK(launch_reduce_f64(ctx->m, ctx->Gpart64, ctx->n_splits, mode, ctx->st));
    }
  }
  else if (ctx->path == PATH_MFMA) CK(launch_reduce_f32(ctx->m, ctx->Gpart, ctx->n_splits, mode, ctx->st));
  else CK(launch_reduce_f64(ctx->m, ctx->Gpart64, ctx->unf_splits, mode, ctx->st));
  return PCV_OK;
}

int split_count(pcv_ctx ctx) {
  return ctx->path == PATH_MFMA || ctx->path == PATH_VALU_SPLIT ? ctx->n_splits : 1;
}

// Value and gradient at q1 into logp1 / g1 (no leapfrog update).
pcv_status eval_q1(pcv_ctx ctx) {
  if (ctx->path == PATH_VALU) {
    CK(launch_valu(ctx->m, ctx->Xv, ctx->fp64, ctx->pb, ctx->W, 1, 0, 0, 0, ctx->st));
    return PCV_OK;
  }
  TRY(split_partials(ctx, true));
  TRY(split_reduce(ctx, 0));
  CK(launch_value_finish(ctx->m, ctx->Vpart, split_count(ctx), ctx->st));
  return PCV_OK;
}

// q0 := q1 state after eval_q1, plus s0.
pcv_status adopt_q1(pcv_ctx ctx) {
  DevModel& m = ctx->m;
  const size_t bytes = sizeof(double) * m.d * m.C;
  CK(hipMemcpyAsync(m.q0, m.q1, bytes, hipMemcpyDeviceToDevice, ctx->st));
  CK(hipMemcpyAsync(m.g0, m.g1, bytes, hipMemcpyDeviceToDevice, ctx->st));
  CK(hipMemcpyAsync(m.logp0, m.logp1, sizeof(double) * m.C, hipMemcpyDeviceToDevice, ctx->st));
  CK(launch_logpred(m, ctx->st));
  return PCV_OK;
}

// One transition of the split paths.  t >= 0: explicit iteration number;
// t < 0: kernels read the device counter, which the last node advances.
pcv_status transition_split(pcv_ctx ctx, int64_t t) {
  DevModel& m = ctx->m;
  CK(launch_momentum(m, t, ctx->st));
  for (int s = 0; s < m.S; ++s) {
    const bool last = s == m.S - 1;
    TRY(split_partials(ctx, last));
    TRY(split_reduce(ctx, last ? 2 : 1));
  }
  if (m.lp_part) CK(launch_testlp(m, ctx->max_test_rows, ctx->st));
  CK(launch_accept(m, ctx->Vpart, split_count(ctx), t, ctx->st));
  if (t < 0) CK(launch_tick(m, ctx->st));
  return PCV_OK;
}

// Capture one transition (device counter mode) into a graph on a private
// stream; replays are launched on the context stream.  The captured work
// holds no memset nodes.  The library GEMMs of the unfused path are not
// captured (that path runs eagerly).
pcv_status capture_transition(pcv_ctx ctx) {
  if (ctx->graph_exec) return PCV_OK;
  if (!ctx->cap_stream) CK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t user = ctx->st;
  ctx->st = ctx->cap_stream;
  const bool timing = ctx->timing;
  ctx->timing = false;
  hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  pcv_status s = PCV_OK;
  if (e == hipSuccess) s = transition_split(ctx, -1);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
  ctx->st = user;
  ctx->timing = timing;
  if (e != hipSuccess || e2 != hipSuccess || s != PCV_OK || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    ctx->graphs = false;   // fall back to eager launches of the same kernels
    return PCV_OK;
  }
  ctx->graph = g;
  CK(hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
  return PCV_OK;
}

// Row ranges [wr[w], wr[w+1]) of the W waves of a fused-VALU workgroup.  For
// the hierarchical family the cuts are moved to group starts so each group
// has one owner wave.
// Even row partition of [lo, hi) over W waves: W + 1 boundaries.  Groups of
// the hierarchical family may straddle wave boundaries (the kernels fold the
// shared groups in a fixed order).
std::vector<int32_t> valu_partition_range(int64_t lo, int64_t hi, int W) {
  std::vector<int32_t> wr(W + 1);
  for (int w = 0; w <= W; ++w) wr[w] = static_cast<int32_t>(lo + (hi - lo) * w / W);
  return wr;
}

std::vector<int32_t> valu_partition(int64_t n, int W) { return valu_partition_range(0, n, W); }

void drop_graph(pcv_ctx ctx);

// Largest row-split count at W waves per workgroup: each wave keeps at least 8 rows.
int valu_split_max_w(pcv_ctx ctx, int W) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(512, ctx->m.n / (8 * W))));
}
int valu_split_max(pcv_ctx ctx) { return valu_split_max_w(ctx, ctx->W); }

// Row-split VALU launch shape as one autotuner config: VALU_CFG_WAVES * W +
// splits, W = 1, 2, 4 or 8 waves per workgroup; a bare split count (below
// VALU_CFG_WAVES) keeps the context's waves.
constexpr int VALU_CFG_WAVES = 1024;
int valu_cfg_waves(pcv_ctx ctx, int cfg) { return cfg >= VALU_CFG_WAVES ? cfg / VALU_CFG_WAVES : ctx->W; }
bool valu_split_cfg_ok(pcv_ctx ctx, int cfg) {
  const int W = valu_cfg_waves(ctx, cfg), ns = cfg % VALU_CFG_WAVES;
  return cfg >= 1 && (W == 1 || W == 2 || W == 4 || W == 8) &&
         valu_smem_bytes(ctx->fp64, W, ctx->m.family, ctx->m.n_groups, ctx->pb) <= 65536 && ns >= 1 &&
         ns <= valu_split_max_w(ctx, W);
}

// Row-split VALU path: ns splits of the rows, W waves each (even
// partitions), the splits spanning each group (hierarchical; rows are sorted
// by group, and a group no split spans gets an empty range), and partial
// buffers [ns][R][C] and [ns][C].
pcv_status apply_valu_splits(pcv_ctx ctx, int ns) {
  DevModel& m = ctx->m;
  const int64_t n = m.n, C = m.C;
  const int W = ctx->W;
  std::vector<int32_t> wr;
  for (int64_t sp = 0; sp < ns; ++sp) {
    const std::vector<int32_t> part = valu_partition_range(n * sp / ns, n * (sp + 1) / ns, W);
    wr.insert(wr.end(), part.begin(), part.end());
  }
  if (wr.size() > ctx->wave_rows_cap) {   // ns x (W + 1) row bounds
    int32_t* d;
    TRY(dalloc(ctx, &d, wr.size()));
    ctx->wave_rows = d;
    ctx->wave_rows_cap = wr.size();
  }
  CK(hipMemcpy(ctx->wave_rows, wr.data(), sizeof(int32_t) * wr.size(), hipMemcpyHostToDevice));
  m.wave_rows = ctx->wave_rows;
  const bool hier = hier_family(m.family);
  if (hier) {
    const int32_t* go = ctx->group_of_host.data();
    std::vector<int32_t> gs(2 * static_cast<size_t>(m.n_groups));
    for (int g = 0; g < m.n_groups; ++g) {
      gs[2 * g] = ns;
      gs[2 * g + 1] = -1;
    }
    for (int64_t sp = 0; sp < ns; ++sp) {
      const int64_t a = n * sp / ns, b = n * (sp + 1) / ns;
      if (b <= a) continue;
      for (int g = go[a]; g <= go[b - 1]; ++g) {
        gs[2 * g] = std::min<int32_t>(gs[2 * g], static_cast<int32_t>(sp));
        gs[2 * g + 1] = std::max<int32_t>(gs[2 * g + 1], static_cast<int32_t>(sp));
      }
    }
    if (!m.gsplit) {
      int32_t* d;
      TRY(dalloc(ctx, &d, gs.size()));
      m.gsplit = d;
    }
    CK(hipMemcpy(const_cast<int32_t*>(m.gsplit), gs.data(), sizeof(int32_t) * gs.size(), hipMemcpyHostToDevice));
  }
  if (hier && !ctx->uscr) TRY(dalloc(ctx, &ctx->uscr, static_cast<size_t>(C)));
  if (ns > ctx->split_cap) {
    double* g;
    double* v;
    TRY(dalloc(ctx, &g, static_cast<size_t>(ns) * m.d * C));
    TRY(dalloc(ctx, &v, static_cast<size_t>(ns) * C));
    ctx->Gpart64 = g;
    ctx->Vpart = v;
    ctx->split_cap = ns;
  }
  ctx->n_splits = ns;
  drop_graph(ctx);
  return PCV_OK;
}
pcv_status apply_valu_split_cfg(pcv_ctx ctx, int cfg) {
  if (!valu_split_cfg_ok(ctx, cfg)) return fail(ctx, PCV_ERR_INVALID_ARG, "invalid row-split launch configuration");
  const int W0 = ctx->W;
  ctx->W = valu_cfg_waves(ctx, cfg);   // the row partition is built for the new waves
  const pcv_status s = apply_valu_splits(ctx, cfg % VALU_CFG_WAVES);
  if (s != PCV_OK) ctx->W = W0;
  return s;
}


bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

extern "C" {

const char* pcv_status_str(pcv_status s) {
  switch (s) {
    case PCV_OK: return "ok";
    case PCV_ERR_INVALID_ARG: return "invalid argument";
    case PCV_ERR_NOMEM: return "out of memory";
    case PCV_ERR_DEVICE: return "device error";
    case PCV_ERR_STATE: return "invalid state";
    case PCV_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* pcv_last_error(pcv_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void pcv_destroy(pcv_ctx ctx) {
  if (!ctx) return;
  if (!ctx->allocs.empty()) {
    if (ctx->st) (void)hipStreamSynchronize(ctx->st);
    else (void)hipDeviceSynchronize();
  }
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->rb) rocblas_destroy_handle(ctx->rb);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

// Scratch memory of pcv_shuffle_benchmark_noalloc: a file-scope device
// array, so that entry point allocates nothing.  Every GPU the library runs
// on holds its own copy until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: the device address
// of this GPU's copy is looked up once per device (with that device
// current) and kept in g_scratch_dev, and only that address reaches kernels.
static __device__ __align__(256) double scratch[PCV_SHUFFLE_NOALLOC_MAX_DOUBLES];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;   // [device] address of its copy, or null

// Resolve (once per device) the current device's copy of the scratch array.
pcv_status resolve_scratch(pcv_ctx ctx) {
  int dev = 0;
  CK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (static_cast<size_t>(dev) >= g_scratch_dev.size()) g_scratch_dev.resize(static_cast<size_t>(dev) + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ctx, PCV_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  ctx->noalloc_scratch = g_scratch_dev[dev];
  return PCV_OK;
}
}  // namespace

namespace {
// MFMA path: switch the gradient kernel's tile shape, packing X for it on
// first use (the fp64 design stays resident for that).
pcv_status apply_mfma_shape(pcv_ctx ctx, int shape) {
  if (!mfma_shape_ok(shape, ctx->m.p))
    return fail(ctx, PCV_ERR_INVALID_ARG, "unknown MFMA shape, or one the design width does not allow");
  const int layout = mfma_layout(shape);   // the two 16x16x32 and the two 32x32x16 kernels share packings
  if (!ctx->Xpk_shape[layout]) {
    const int p = static_cast<int>(ctx->m.p);
    const size_t nfr = static_cast<size_t>(ctx->n_tiles) * mfma_nfrag(p, shape) * 64;
    uint4* xp;
    TRY(dalloc(ctx, &xp, nfr));
    CK(launch_mfma_pack(ctx->m.X64, ctx->m.n, p, ctx->n_tiles, shape, xp, ctx->st));
    ctx->Xpk_shape[layout] = xp;
  }
  ctx->Xpk = ctx->Xpk_shape[layout];
  ctx->mshape = shape;
  drop_graph(ctx);
  return PCV_OK;
}
}  // namespace

static pcv_status init_impl(pcv_ctx ctx, const pcv_model* md, const double* X, const double* y,
                            const pcv_folds* fm) {
  if (!md || !X || !y || !fm) return fail(ctx, PCV_ERR_INVALID_ARG, "null argument");
  const int64_t n = md->n, p = md->p;
  if (n <= 0 || p <= 0 || md->K <= 0) return fail(ctx, PCV_ERR_INVALID_ARG, "n, p and K must be positive");
  if (md->L < 2 || md->L > 64) return fail(ctx, PCV_ERR_INVALID_ARG, "L must be in [2, 64]");
  if (md->family < 0 || md->family > 4) return fail(ctx, PCV_ERR_INVALID_ARG, "unknown family");
  if (md->precision < 0 || md->precision > 4) return fail(ctx, PCV_ERR_INVALID_ARG, "unknown precision");
  if (md->x_format != PCV_X_FP64 && md->x_format != PCV_X_BF16_HILO)
    return fail(ctx, PCV_ERR_INVALID_ARG, "unknown x_format");
  if (md->rhat_mode != PCV_RHAT_WELFORD && md->rhat_mode != PCV_RHAT_SHIFTED_SUMS)
    return fail(ctx, PCV_ERR_INVALID_ARG, "unknown rhat_mode");
  if (md->scores < 0 || md->scores > (PCV_SCORE_HS | PCV_SCORE_DSS))
    return fail(ctx, PCV_ERR_INVALID_ARG, "unknown scores");
  if (md->store_draws < 0) return fail(ctx, PCV_ERR_INVALID_ARG, "store_draws must be >= 0");
  if ((md->scores & PCV_SCORE_HS) && md->family != PCV_FAMILY_GAUSSIAN)
    return fail(ctx, PCV_ERR_UNSUPPORTED, "the Hyvarinen score needs a continuous response (Gaussian family)");
  if (!(md->step_size > 0) || !std::isfinite(md->step_size)) return fail(ctx, PCV_ERR_INVALID_ARG, "step_size must be > 0");
  if (md->n_leapfrog < 1) return fail(ctx, PCV_ERR_INVALID_ARG, "n_leapfrog must be >= 1");
  if (md->batch_size < 1 || md->batches_per_block < 1 || md->n_blocks < 1 || md->n_blocks > MAX_BLOCKS)
    return fail(ctx, PCV_ERR_INVALID_ARG, "batch_size, batches_per_block >= 1 and 1 <= n_blocks <= 64 required");
  if (md->n_warmup < 0 || md->chain_offset < 0) return fail(ctx, PCV_ERR_INVALID_ARG, "negative n_warmup or chain_offset");
  const bool hier = md->family == PCV_FAMILY_HIER_LOGISTIC || md->family == PCV_FAMILY_HIER_GAUSSIAN;
  const bool hgauss = md->family == PCV_FAMILY_HIER_GAUSSIAN;
  if (hier && (md->n_groups <= 0 || !md->group_of)) return fail(ctx, PCV_ERR_INVALID_ARG, "hierarchical family needs groups");
  const int64_t d = hier ? p + (hgauss ? 3 : 2) + md->n_groups : p;
  if (hgauss && md->scores)
    return fail(ctx, PCV_ERR_UNSUPPORTED, "HS and DSS are not built for the hierarchical Gaussian family");
  // models in one launch (Appendix B): M x K posteriors, model-major
  const int M = md->n_models > 1 ? md->n_models : 1;
  if (md->n_models < 0) return fail(ctx, PCV_ERR_INVALID_ARG, "n_models must be >= 0");
  if (M > 1) {
    if (!md->model_mask) return fail(ctx, PCV_ERR_INVALID_ARG, "n_models > 1 needs model_mask");
    for (int64_t i = 0; i < static_cast<int64_t>(M) * p; ++i)
      if (md->model_mask[i] > 1) return fail(ctx, PCV_ERR_INVALID_ARG, "model_mask entries must be 0 or 1");
    if (hier && md->precision != PCV_PREC_FP64 && md->precision != PCV_PREC_FP32)
      return fail(ctx, PCV_ERR_UNSUPPORTED, "several hierarchical models in one launch: fp64 and fp32 paths");
    if (md->scores) return fail(ctx, PCV_ERR_UNSUPPORTED, "several models in one launch: no scores");
    if (md->precision == PCV_PREC_FP64_UNFUSED)
      return fail(ctx, PCV_ERR_UNSUPPORTED, "several models in one launch: not on the plain fp64 path");
  }
  const int64_t C = static_cast<int64_t>(M) * md->K * md->L;
  if (md->chain_offset + C > 0xFFFFFFFFLL) return fail(ctx, PCV_ERR_INVALID_ARG, "global chain ids must fit 32 bits");
  if (!md->inv_mass || !md->init_pos) return fail(ctx, PCV_ERR_INVALID_ARG, "inv_mass and init_pos are required");
  if (md->family == PCV_FAMILY_GAUSSIAN && !(md->sigma > 0 && std::isfinite(md->sigma)))
    return fail(ctx, PCV_ERR_INVALID_ARG, "sigma must be > 0");
  if (!finite_all(X, n * p) || !finite_all(y, n)) return fail(ctx, PCV_ERR_INVALID_ARG, "X and y must be finite");
  if (!finite_all(md->init_pos, C * d)) return fail(ctx, PCV_ERR_INVALID_ARG, "init_pos must be finite");
  for (int64_t j = 0; j < d; ++j)
    if (!(md->inv_mass[j] > 0) || !std::isfinite(md->inv_mass[j]))
      return fail(ctx, PCV_ERR_INVALID_ARG, "inv_mass must be > 0");
  if (md->prior_scale && !hier)
    for (int64_t j = 0; j < d; ++j)
      if (!(md->prior_scale[j] > 0) || !std::isfinite(md->prior_scale[j]))
        return fail(ctx, PCV_ERR_INVALID_ARG, "prior_scale must be > 0");
  for (int64_t i = 0; i < n; ++i) {
    const double v = y[i];
    if ((md->family == PCV_FAMILY_LOGISTIC || md->family == PCV_FAMILY_HIER_LOGISTIC) && !(v == 0.0 || v == 1.0))
      return fail(ctx, PCV_ERR_INVALID_ARG, "Bernoulli responses must be 0 or 1");
    if (md->family == PCV_FAMILY_POISSON && !(v >= 0.0 && v == std::floor(v)))
      return fail(ctx, PCV_ERR_INVALID_ARG, "Poisson responses must be non-negative integers");
  }
  if (hier) {
    for (int64_t i = 0; i < n; ++i) {
      const int g = md->group_of[i];
      if (g < 0 || g >= md->n_groups || (i > 0 && g < md->group_of[i - 1]))
        return fail(ctx, PCV_ERR_INVALID_ARG, "group_of must be sorted and in [0, n_groups)");
    }
  }

  // ---- folds: validate, count, build the test-row lists ------------------
  const int K = md->K;
  std::vector<int32_t> test_ptr(K + 1, 0), test_rows;
  std::vector<int64_t> train_cnt(K, 0);
  std::vector<int32_t> ivals;
  if (fm->kind == PCV_FOLDS_INDEX) {
    if (!fm->fold_index) return fail(ctx, PCV_ERR_INVALID_ARG, "fold_index missing");
    for (int64_t i = 0; i < n; ++i) {
      const int f = fm->fold_index[i];
      if (f < -1 || f >= K) return fail(ctx, PCV_ERR_INVALID_ARG, "fold_index out of range");
      if (f >= 0) test_ptr[f + 1]++;
    }
    for (int k = 0; k < K; ++k) train_cnt[k] = n - test_ptr[k + 1];
    for (int k = 0; k < K; ++k) test_ptr[k + 1] += test_ptr[k];
    test_rows.resize(test_ptr[K]);
    std::vector<int32_t> fill(test_ptr.begin(), test_ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      if (fm->fold_index[i] >= 0) test_rows[fill[fm->fold_index[i]]++] = static_cast<int32_t>(i);
  } else if (fm->kind == PCV_FOLDS_INTERVALS) {
    if (!fm->intervals) return fail(ctx, PCV_ERR_INVALID_ARG, "intervals missing");
    if (n > 0x7FFFFFFF) return fail(ctx, PCV_ERR_INVALID_ARG, "n too large for intervals");
    ivals.resize(4 * K);
    for (int k = 0; k < K; ++k) {
      const int64_t* v = fm->intervals + 4 * k;
      if (v[0] < 0 || v[1] < v[0] || v[1] > n || v[2] < 0 || v[3] < v[2] || v[3] > n)
        return fail(ctx, PCV_ERR_INVALID_ARG, "intervals out of range");
      // The kernels take a fold's non-train rows as one range: store the hull
      // of the test and excluded ranges, which must touch or overlap when
      // both are non-empty.
      int64_t nlo = v[2], nhi = v[3];
      if (v[1] > v[0]) {
        if (v[3] > v[2] && (v[1] < v[2] || v[3] < v[0]))
          return fail(ctx, PCV_ERR_INVALID_ARG, "intervals: test and excluded ranges of a fold must overlap or touch");
        nlo = v[3] > v[2] ? std::min(v[0], v[2]) : v[0];
        nhi = v[3] > v[2] ? std::max(v[1], v[3]) : v[1];
      }
      ivals[4 * k + 0] = static_cast<int32_t>(v[0]);
      ivals[4 * k + 1] = static_cast<int32_t>(v[1]);
      ivals[4 * k + 2] = static_cast<int32_t>(nlo);
      ivals[4 * k + 3] = static_cast<int32_t>(nhi);
      for (int64_t i = v[0]; i < v[1]; ++i) test_rows.push_back(static_cast<int32_t>(i));
      test_ptr[k + 1] = static_cast<int32_t>(test_rows.size());
      train_cnt[k] = n - (nhi - nlo);
    }
  } else if (fm->kind == PCV_FOLDS_DENSE) {
    if (!fm->roles) return fail(ctx, PCV_ERR_INVALID_ARG, "roles missing");
    for (int k = 0; k < K; ++k) {
      for (int64_t i = 0; i < n; ++i) {
        const int r = fm->roles[static_cast<int64_t>(k) * n + i];
        if (r < 0 || r > 2) return fail(ctx, PCV_ERR_INVALID_ARG, "roles must be 0, 1 or 2");
        if (r == 2) test_rows.push_back(static_cast<int32_t>(i));
        if (r == 1) train_cnt[k]++;
      }
      test_ptr[k + 1] = static_cast<int32_t>(test_rows.size());
    }
  } else {
    return fail(ctx, PCV_ERR_INVALID_ARG, "unknown fold encoding");
  }
  for (int k = 0; k < K; ++k) {
    // a single fold without test rows is the full-data model (s = 0), the
    // context that pcv_adapt tunes
    if (test_ptr[k + 1] == test_ptr[k] && K > 1) return fail(ctx, PCV_ERR_INVALID_ARG, "a fold has no test row");
    if (train_cnt[k] <= 0) return fail(ctx, PCV_ERR_INVALID_ARG, "a fold has no training row");
  }

  // ---- path selection ------------------------------------------------------
  ctx->prec = md->precision;
  {
    uint64_t h = 0xcbf29ce484222325ULL;
    h = fp_mix(h, X, sizeof(double) * static_cast<size_t>(n * p));
    h = fp_mix(h, y, sizeof(double) * static_cast<size_t>(n));
    if (fm->kind == PCV_FOLDS_INDEX) h = fp_mix(h, fm->fold_index, sizeof(int32_t) * static_cast<size_t>(n));
    if (fm->kind == PCV_FOLDS_INTERVALS) h = fp_mix(h, fm->intervals, sizeof(int64_t) * 4 * static_cast<size_t>(K));
    if (fm->kind == PCV_FOLDS_DENSE) h = fp_mix(h, fm->roles, static_cast<size_t>(K) * static_cast<size_t>(n));
    if (hier) h = fp_mix(h, md->group_of, sizeof(int32_t) * static_cast<size_t>(n));
    if (M > 1) {
      const int64_t mm = M;
      h = fp_mix(h, &mm, sizeof mm);
      h = fp_mix(h, md->model_mask, static_cast<size_t>(M) * static_cast<size_t>(p));
    }
    ctx->fingerprint = h;
    uint64_t f = 0xcbf29ce484222325ULL;
    const int64_t shape[3] = {fm->kind, n, K};
    f = fp_mix(f, shape, sizeof shape);
    if (fm->kind == PCV_FOLDS_INDEX) f = fp_mix(f, fm->fold_index, sizeof(int32_t) * static_cast<size_t>(n));
    if (fm->kind == PCV_FOLDS_INTERVALS) f = fp_mix(f, fm->intervals, sizeof(int64_t) * 4 * static_cast<size_t>(K));
    if (fm->kind == PCV_FOLDS_DENSE) f = fp_mix(f, fm->roles, static_cast<size_t>(K) * static_cast<size_t>(n));
    ctx->fold_fp = f;
  }
  if (md->precision == PCV_PREC_FP64 || md->precision == PCV_PREC_FP32) {
    ctx->path = PATH_VALU;
    ctx->fp64 = md->precision == PCV_PREC_FP64;
    ctx->pb = valu_pb(p, ctx->fp64);
    if (!ctx->pb) return fail(ctx, PCV_ERR_UNSUPPORTED, "VALU paths support p <= 64");
    // few chains and many rows: split rows across workgroups (partial sums
    // reduced per leapfrog step) instead of one fused workgroup per 64 chains
    const int64_t chain_blocks = (C + 63) / 64;
    if (chain_blocks < 128 && n >= 2048) ctx->path = PATH_VALU_SPLIT;
  } else if (md->precision == PCV_PREC_BF16X3 || md->precision == PCV_PREC_BF16X5) {
    ctx->path = PATH_MFMA;
    ctx->fwd = md->precision == PCV_PREC_BF16X5 ? 5 : 3;
    if (hier) return fail(ctx, PCV_ERR_UNSUPPORTED, "bf16 MFMA path supports the GLM families");
    if (p > 128) return fail(ctx, PCV_ERR_UNSUPPORTED, "bf16 MFMA path supports p <= 128");
    if (fm->kind == PCV_FOLDS_DENSE)
      return fail(ctx, PCV_ERR_UNSUPPORTED, "bf16 MFMA path takes index or interval fold encodings");
  } else {
    ctx->path = PATH_UNFUSED;
    if (hier) return fail(ctx, PCV_ERR_UNSUPPORTED, "unfused fp64 path supports the GLM families");
  }

  // ---- model constants ---------------------------------------------------
  DevModel& m = ctx->m;
  m.family = md->family;
  m.fold_kind = fm->kind;
  m.n = n;
  m.p = p;
  m.d = d;
  m.C = C;
  m.K = K;
  m.M = M;
  m.KP = M * K;
  m.L = md->L;
  m.n_groups = hier ? md->n_groups : 0;
  m.sigma = md->family == PCV_FAMILY_GAUSSIAN ? md->sigma : 1.0;
  m.inv_sigma2 = 1.0 / (m.sigma * m.sigma);
  m.eps = md->step_size;
  m.S = md->n_leapfrog;
  m.n_warmup = md->n_warmup;
  m.rhat_mode = md->rhat_mode;
  m.b = md->batch_size;
  m.Gb = md->batches_per_block;
  m.D = md->n_blocks;
  m.key0 = static_cast<uint32_t>(md->seed & 0xFFFFFFFFu);
  m.key1 = static_cast<uint32_t>(md->seed >> 32);
  m.chain_offset = md->chain_offset;

  std::vector<double> prior_prec(d, 1.0);
  double prior_const = 0.0;
  const double half_log_2pi = 0.5 * std::log(2.0 * M_PI);
  if (hgauss) {
    // beta, mu, z standard normal; sigma_a, sigma_y half-normal with variance
    // HGAUSS_SCALE_VAR (their log-Jacobians and exponents are in prior_quad)
    prior_const = -static_cast<double>(d - 2) * half_log_2pi +
                  2.0 * (std::log(2.0) - 0.5 * std::log(2.0 * M_PI * HGAUSS_SCALE_VAR));
  } else if (hier) {
    prior_const = -static_cast<double>(d - 1) * half_log_2pi + (std::log(2.0) - half_log_2pi);
  } else {
    for (int64_t j = 0; j < d; ++j) {
      const double s = md->prior_scale ? md->prior_scale[j] : 1.0;
      prior_prec[j] = 1.0 / (s * s);
      prior_const += -half_log_2pi - std::log(s);
    }
  }
  ctx->prior_const = prior_const;
  // the target density belongs to the checkpoint fingerprint too: a run
  // resumes only under the same noise scale and prior
  ctx->fingerprint = fp_mix(ctx->fingerprint, &m.sigma, sizeof(double));
  ctx->fingerprint = fp_mix(ctx->fingerprint, prior_prec.data(), sizeof(double) * static_cast<size_t>(d));

  // ---- device data -------------------------------------------------------
  double *X64, *y64, *minv, *pprec, *rowc, *fconst;
  // first device work: everything above only validated the host arguments
  TRY(resolve_scratch(ctx));
  TRY(upload(ctx, &X64, X, n * p));
  TRY(upload(ctx, &y64, y, n));
  TRY(upload(ctx, &minv, md->inv_mass, d));
  TRY(upload(ctx, &pprec, prior_prec.data(), d));
  TRY(dalloc(ctx, &rowc, n));
  TRY(dalloc(ctx, &fconst, K));
  if (M > 1) {
    uint8_t* mk;
    TRY(upload(ctx, &mk, md->model_mask, static_cast<size_t>(M) * static_cast<size_t>(p)));
    m.mmask = mk;
  }
  std::vector<float> y32(y, y + n);
  float* y32d;
  TRY(upload(ctx, &y32d, y32.data(), n));
  m.X64 = X64;
  m.y64 = y64;
  m.y32 = y32d;
  m.minv = minv;
  m.prior_prec = pprec;
  m.rowc = rowc;
  m.fold_const = fconst;
  {
    std::vector<double> ntr(train_cnt.begin(), train_cnt.end());
    double* nt;
    TRY(upload(ctx, &nt, ntr.data(), ntr.size()));
    m.ntrain = nt;
  }
  int32_t *tp, *tr;
  TRY(upload(ctx, &tp, test_ptr.data(), test_ptr.size()));
  TRY(upload(ctx, &tr, test_rows.data(), test_rows.size()));
  m.test_ptr = tp;
  m.test_rows = tr;
  m.scores = md->scores;
  ctx->test_ptr_host = test_ptr;
  for (int k = 0; k < K; ++k) ctx->max_test_rows = std::max(ctx->max_test_rows, test_ptr[k + 1] - test_ptr[k]);
  // The proposal's test-row log predictive gets a kernel of its own (spread
  // over test rows as well as chains) when the accept kernel's workgroups
  // (one per 64 chains) are fewer than the CUs and a chain's share is long
  // enough to pay for the extra launch.  Measured per transition: 4000 and
  // 800 chains with 40 x 64 and 200 x 10 (rows x coefficients) gain 3-8%;
  // 8000 chains with 5 x 4 lose 3%; 40000 chains with 10 x 128 lose 0.1%
  // (their accept kernel already fills the chip).
  // (k_testlp stages a block's coefficients in LDS: designs of up to 128.)
  if (static_cast<int64_t>(ctx->max_test_rows) * p > 512 && (C + 63) / 64 < 256 && p <= 128) {
    m.lp_groups = testlp_groups(ctx->max_test_rows);
    TRY(dalloc(ctx, &m.lp_part, static_cast<size_t>(m.lp_groups) * static_cast<size_t>(C)));
  }
  if (md->store_draws > 0) {
    TRY(dalloc(ctx, &m.draws, static_cast<size_t>(md->store_draws) * static_cast<size_t>(C)));
    m.draws_cap = md->store_draws;
  }
  if (md->scores) {
    const size_t nnz = static_cast<size_t>(test_ptr[K]);
    std::vector<int64_t> sq(K + 1, 0);
    for (int k = 0; k < K; ++k) {
      const int64_t v = test_ptr[k + 1] - test_ptr[k];
      sq[k + 1] = sq[k] + v * v;
    }
    ctx->sq_ptr_host = sq;
    const size_t Lz = static_cast<size_t>(md->L);
    if (md->scores & PCV_SCORE_HS) {
      TRY(dalloc(ctx, &m.hs1, static_cast<size_t>(C)));
      TRY(dalloc(ctx, &m.hs2, Lz * nnz));
    }
    if (md->scores & PCV_SCORE_DSS) {
      TRY(dalloc(ctx, &m.dx, Lz * nnz));
      TRY(dalloc(ctx, &m.rcur, Lz * nnz));
      TRY(dalloc(ctx, &m.dxx, Lz * static_cast<size_t>(sq[K])));
      int64_t* sqd;
      TRY(upload(ctx, &sqd, sq.data(), sq.size()));
      m.sq_ptr = sqd;
    }
  }
  if (fm->kind == PCV_FOLDS_INDEX) {
    int32_t* fi;
    TRY(upload(ctx, &fi, fm->fold_index, n));
    m.fold_index = fi;
  } else if (fm->kind == PCV_FOLDS_INTERVALS) {
    int32_t* iv;
    TRY(upload(ctx, &iv, ivals.data(), ivals.size()));
    m.ivals = iv;
  } else {
    int8_t* rl;
    TRY(upload(ctx, &rl, fm->roles, static_cast<size_t>(K) * n));
    m.roles = rl;
  }
  if (hier) {
    int32_t* go;
    TRY(upload(ctx, &go, md->group_of, n));
    m.group_of = go;
  }

  // chain state and accumulators
  const size_t dc = static_cast<size_t>(d) * C;
  TRY(dalloc(ctx, &m.q0, dc));
  TRY(dalloc(ctx, &m.g0, dc));
  TRY(dalloc(ctx, &m.q1, dc));
  TRY(dalloc(ctx, &m.g1, dc));
  TRY(dalloc(ctx, &m.pm, dc));
  TRY(dalloc(ctx, &m.logp0, C));
  TRY(dalloc(ctx, &m.logp1, C));
  TRY(dalloc(ctx, &m.s0, C));
  TRY(dalloc(ctx, &m.h0, C));
  TRY(dalloc(ctx, &m.Z, C));
  TRY(dalloc(ctx, &m.U, C));
  TRY(dalloc(ctx, &m.U2, C));
  TRY(dalloc(ctx, &m.V, C));
  TRY(dalloc(ctx, &m.V2, C));
  TRY(dalloc(ctx, &m.bmean, static_cast<size_t>(m.D) * C));
  TRY(dalloc(ctx, &m.bm2, static_cast<size_t>(m.D) * C));
  TRY(dalloc(ctx, &m.nacc, C));
  TRY(dalloc(ctx, &m.ndiv, C));
  TRY(dalloc(ctx, &m.wsum, C));
  TRY(dalloc(ctx, &m.center, static_cast<size_t>(m.KP)));
  TRY(dalloc(ctx, &m.t_dev, 1));
  TRY(dalloc(ctx, &m.acc_stat, C));
  TRY(dalloc(ctx, &ctx->fold_buf, 6 * static_cast<size_t>(m.KP)));
  TRY(dalloc(ctx, &ctx->dscal, 8));
  TRY(dalloc(ctx, &ctx->Vpart, C));

  // ---- path-specific buffers -----------------------------------------------
  if (ctx->path == PATH_VALU || ctx->path == PATH_VALU_SPLIT) {
    const int pb = ctx->pb;
    const int64_t npad = n;
    if (ctx->fp64) {
      std::vector<double> xv(static_cast<size_t>(npad) * pb, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < p; ++j) xv[i * pb + j] = X[i * p + j];
      double* xd;
      TRY(upload(ctx, &xd, xv.data(), xv.size()));
      ctx->Xv = xd;
    } else {
      std::vector<float> xv(static_cast<size_t>(npad) * pb, 0.f);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < p; ++j) xv[i * pb + j] = static_cast<float>(X[i * p + j]);
      float* xd;
      TRY(upload(ctx, &xd, xv.data(), xv.size()));
      ctx->Xv = xd;
      m.X32 = xd;
    }
    // Autoregressive designs: every row after the first holds the previous
    // row's response followed by the previous row's first p - 1 coefficients
    // (exact equality), so the row-split kernel slides them in registers.
    if (ctx->path == PATH_VALU_SPLIT && !hier && pb == p && n >= 2) {
      bool lag = true;
      for (int64_t i = 1; i < n && lag; ++i) {
        lag = X[i * p] == y[i - 1];
        for (int64_t j = 1; j < p && lag; ++j) lag = X[i * p + j] == X[(i - 1) * p + j - 1];
      }
      ctx->series = lag;
    }
    if (ctx->path == PATH_VALU_SPLIT) {
      // W waves per workgroup, row splits so that (chain blocks x splits)
      // fills the GPU several times over while each wave keeps >= 32 rows
      int W = 4;
      while (W > 1 && valu_smem_bytes(ctx->fp64, W, m.family, m.n_groups, ctx->pb) > 65536) --W;
      if (valu_smem_bytes(ctx->fp64, W, m.family, m.n_groups, ctx->pb) > 65536)
        return fail(ctx, PCV_ERR_UNSUPPORTED, "too many groups for the row-split path");
      // Split count: workgroups run in rounds of (compute units x resident
      // workgroups per unit); a workgroup costs its rows per wave plus about
      // 32 rows' worth of set-up and partial-sum traffic.  Pick the count
      // with the smallest rounds x cost (the fewest splits among ties).
      const int64_t chain_blocks = (C + 63) / 64;
      int dev = 0, cus = 0;
      CK(hipGetDevice(&dev));
      CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      const int bpc = std::max(1, valu_part_occupancy(ctx->fp64, m.family, ctx->pb, W,
                                                      valu_smem_bytes(ctx->fp64, W, m.family, m.n_groups, ctx->pb)));
      const int64_t cap = static_cast<int64_t>(std::max(1, cus)) * bpc;
      int64_t ns = 1;
      double best = 1e300;
      ctx->W = W;
      for (int64_t cand = 1; cand <= valu_split_max(ctx); ++cand) {
        const double rounds = static_cast<double>((chain_blocks * cand + cap - 1) / cap);
        const double cost = rounds * (std::ceil(static_cast<double>(n) / static_cast<double>(cand * W)) + 32.0);
        if (cost < best - 1e-9) {
          best = cost;
          ns = cand;
        }
      }
      ctx->W = W;
      if (hier) ctx->group_of_host.assign(md->group_of, md->group_of + n);
      TRY(apply_valu_splits(ctx, static_cast<int>(ns)));
    } else {
    // waves per workgroup: enough rows per wave, LDS within 64 KB, and the
    // register budget of wide rows.
    int W = static_cast<int>(std::min<int64_t>(8, std::max<int64_t>(1, n / 64)));
    if (pb >= 32) W = std::min(W, 4);
    while (W > 1 && valu_smem_bytes(ctx->fp64, W, m.family, m.n_groups, ctx->pb) > 65536) --W;
    if (valu_smem_bytes(ctx->fp64, W, m.family, m.n_groups, ctx->pb) > 65536)
      return fail(ctx, PCV_ERR_UNSUPPORTED, "too many groups for the fused path");
    ctx->W = W;
    const std::vector<int32_t> wr = valu_partition(n, W);
    TRY(dalloc(ctx, &ctx->wave_rows, 9));   // room for any W <= 8 (autotuning)
    CK(hipMemcpy(ctx->wave_rows, wr.data(), sizeof(int32_t) * wr.size(), hipMemcpyHostToDevice));
    m.wave_rows = ctx->wave_rows;
    }
  } else if (ctx->path == PATH_MFMA) {
    const int R = mfma_rows_per_tile();
    ctx->n_tiles = static_cast<int>((n + R - 1) / R);
    const int ct0 = mfma_chain_tile(MFMA_SHAPE_16X16X32);
    const int n_ct = static_cast<int>((C + ct0 - 1) / ct0);
    // Row splits per chain tile.  One workgroup fits per CU (LDS ring and
    // registers), so workgroups run in rounds of 256; a task costs its tiles
    // plus about four tiles of pipeline fill and partial-result traffic.
    // Pick the split count with the smallest estimated time.
    int ns = 1;
    double best = 1e300;
    for (int cand = 1; cand <= 64 && cand <= ctx->n_tiles; ++cand) {
      const int64_t tasks = static_cast<int64_t>(n_ct) * cand;
      const double rounds = static_cast<double>((tasks + 255) / 256);
      const double per_task = std::ceil(static_cast<double>(ctx->n_tiles) / cand) + 4.0;
      const double cost = rounds * per_task;
      if (cost < best - 1e-9) {
        best = cost;
        ns = cand;
      }
    }
    ctx->tiles_per_split = (ctx->n_tiles + ns - 1) / ns;
    ctx->n_splits = (ctx->n_tiles + ctx->tiles_per_split - 1) / ctx->tiles_per_split;
    if (ctx->tiles_per_split < 1 || static_cast<int64_t>(ctx->n_splits) * ctx->tiles_per_split < ctx->n_tiles)
      return fail(ctx, PCV_ERR_DEVICE, "internal error: row splits do not cover the rows");
    TRY(apply_mfma_shape(ctx, MFMA_SHAPE_32X32X16));
    // per (tile, chain tile): bit w set when a chain of wave w has a
    // non-train row in the tile, or the tile holds padded rows (past n);
    // those waves take the masked epilogue
    {
      // (k_mfma32's workgroups own 256 chains, like k_mfma's, and only they read the flags)
      const int cpw = ct0 / 8;   // chains per wave
      std::vector<uint32_t> fl(static_cast<size_t>(ctx->n_tiles) * n_ct, 0u);
      if (n % R != 0)
        for (int c = 0; c < n_ct; ++c) fl[static_cast<size_t>(ctx->n_tiles - 1) * n_ct + c] = 0xFFu;
      for (int kp = 0; kp < M * K; ++kp) {
        const int k = kp % K;
        std::vector<int> tiles;
        if (fm->kind == PCV_FOLDS_INTERVALS) {
          const int64_t lo = ivals[4 * k + 2], hi = ivals[4 * k + 3];
          for (int64_t t = lo / R; hi > lo && t <= (hi - 1) / R; ++t) tiles.push_back(static_cast<int>(t));
        } else {
          for (int32_t q = test_ptr[k]; q < test_ptr[k + 1]; ++q) tiles.push_back(test_rows[q] / R);
        }
        for (int64_t c = static_cast<int64_t>(kp) * md->L; c < static_cast<int64_t>(kp + 1) * md->L; ++c) {
          const int cti = static_cast<int>(c / ct0);
          const uint32_t bit = 1u << static_cast<int>((c % ct0) / cpw);
          for (int t : tiles) fl[static_cast<size_t>(t) * n_ct + cti] |= bit;
        }
      }
      TRY(upload(ctx, &ctx->tflag, fl.data(), fl.size()));
    }
    std::vector<float> ty(static_cast<size_t>(ctx->n_tiles) * R, 0.f);
    std::vector<int32_t> tf(static_cast<size_t>(ctx->n_tiles) * R, -2);
    for (int64_t i = 0; i < n; ++i) {
      ty[i] = static_cast<float>(y[i]);
      tf[i] = fm->kind == PCV_FOLDS_INDEX ? fm->fold_index[i] : -2;
    }
    TRY(upload(ctx, &ctx->ty, ty.data(), ty.size()));
    TRY(upload(ctx, &ctx->tfid, tf.data(), tf.size()));
    TRY(dalloc(ctx, &ctx->Gpart, static_cast<size_t>(ctx->n_splits) * p * C));
    double* vp;
    TRY(dalloc(ctx, &vp, static_cast<size_t>(ctx->n_splits) * C));
    ctx->Vpart = vp;
    ctx->split_cap = ctx->n_splits;
  } else {
    if (rocblas_create_handle(&ctx->rb) != rocblas_status_success)
      return fail(ctx, PCV_ERR_DEVICE, "rocblas_create_handle failed");
    rocblas_set_stream(ctx->rb, ctx->st);
    ctx->chunk = std::max<int64_t>(1, std::min<int64_t>(C, (int64_t{1} << 28) / n));
    TRY(dalloc(ctx, &ctx->eta, static_cast<size_t>(n) * ctx->chunk));
    {
      // adjoint row splits: about 256 output tiles of 128 x 128 per chunk
      const int64_t tiles = ((ctx->chunk + 127) / 128) * ((p + 127) / 128);
      const int64_t want = std::max<int64_t>(1, std::min<int64_t>({64, 256 / std::max<int64_t>(1, tiles), n}));
      ctx->unf_rows = (n + want - 1) / want;
      const int64_t full = n / ctx->unf_rows;
      ctx->unf_splits = static_cast<int>(full + (n - full * ctx->unf_rows > 0 ? 1 : 0));
    }
    TRY(dalloc(ctx, &ctx->Gpart64, dc * ctx->unf_splits));
    TRY(dalloc(ctx, &ctx->theta_cd, static_cast<size_t>(C) * p));
  }

  // ---- constants, initial state ------------------------------------------
  CK(launch_rowconst(m, rowc, ctx->st));
  CK(launch_foldconst(m, prior_const, fconst, ctx->st));
  double* init_cd;
  TRY(upload(ctx, &init_cd, md->init_pos, dc));
  CK(launch_to_dc(init_cd, m.q1, C, d, ctx->st));
  TRY(eval_q1(ctx));
  TRY(adopt_q1(ctx));
  CK(launch_fill(m.Z, -INFINITY, C, ctx->st));
  CK(launch_fill(m.U, -INFINITY, C, ctx->st));
  CK(launch_fill(m.U2, -INFINITY, C, ctx->st));
  CK(launch_fill(m.V, -INFINITY, C, ctx->st));
  CK(launch_fill(m.V2, -INFINITY, C, ctx->st));
  CK(launch_fill(m.bmean, 0.0, static_cast<int64_t>(m.D) * C, ctx->st));
  CK(launch_fill(m.bm2, 0.0, static_cast<int64_t>(m.D) * C, ctx->st));
  CK(launch_fill(m.wsum, 0.0, C, ctx->st));
  CK(launch_fill(m.center, 0.0, m.KP, ctx->st));
  if (m.hs1) CK(launch_fill(m.hs1, 0.0, C, ctx->st));
  if (m.hs2) CK(launch_fill(m.hs2, 0.0, static_cast<int64_t>(m.L) * ctx->test_ptr_host[K], ctx->st));
  if (m.dx) CK(launch_fill(m.dx, 0.0, static_cast<int64_t>(m.L) * ctx->test_ptr_host[K], ctx->st));
  if (m.dxx) CK(launch_fill(m.dxx, 0.0, static_cast<int64_t>(m.L) * ctx->sq_ptr_host[K], ctx->st));
  CK(hipMemsetAsync(m.nacc, 0, sizeof(int64_t) * C, ctx->st));
  CK(hipMemsetAsync(m.ndiv, 0, sizeof(int64_t) * C, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  return PCV_OK;
}

pcv_status pcv_init(pcv_ctx* out, const pcv_model* model, const void* X, const double* y,
                    const pcv_folds* fold_masks) {
  if (!out) return PCV_ERR_INVALID_ARG;
  *out = nullptr;
  pcv_ctx ctx = new (std::nothrow) pcv_ctx_s();
  if (!ctx) return PCV_ERR_NOMEM;
  // a design given as two bf16 planes is summed (exactly) into fp64 here
  std::vector<double> x_sum;
  const double* X64 = static_cast<const double*>(X);
  pcv_status s = PCV_OK;
  if (model && X && model->x_format == PCV_X_BF16_HILO) {
    if (model->n <= 0 || model->p <= 0 || model->n > (int64_t{1} << 40) / model->p) {
      s = fail(ctx, PCV_ERR_INVALID_ARG, "n and p must be positive");
    } else {
      const size_t np = static_cast<size_t>(model->n * model->p);
      const uint16_t* hi = static_cast<const uint16_t*>(X);
      const uint16_t* lo = hi + np;
      auto bf = [](uint16_t b) {
        const uint32_t u = static_cast<uint32_t>(b) << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return static_cast<double>(f);
      };
      try {
        x_sum.resize(np);
      } catch (...) {
        s = fail(ctx, PCV_ERR_NOMEM, "host memory for X");
      }
      if (s == PCV_OK) {
        for (size_t i = 0; i < np; ++i) x_sum[i] = bf(hi[i]) + bf(lo[i]);
        X64 = x_sum.data();
      }
    }
  }
  if (s == PCV_OK) s = init_impl(ctx, model, X64, y, fold_masks);
  if (s != PCV_OK) {
    // keep the message available through a static copy: the context dies here
    static thread_local std::string last;
    last = ctx->err;
    std::fprintf(stderr, "pcv_init: %s: %s\n", pcv_status_str(s), last.c_str());
    pcv_destroy(ctx);
    return s;
  }
  *out = ctx;
  return PCV_OK;
}

pcv_status pcv_set_stream(pcv_ctx ctx, void* hip_stream) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  ctx->st = static_cast<hipStream_t>(hip_stream);
  if (ctx->rb) rocblas_set_stream(ctx->rb, ctx->st);
  return PCV_OK;
}

static pcv_status step_run(pcv_ctx ctx, int64_t n_iter);

pcv_status pcv_step(pcv_ctx ctx, int64_t n_iter) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (n_iter < 0) return fail(ctx, PCV_ERR_INVALID_ARG, "n_iter must be >= 0");
  if (ctx->t + n_iter > 0xFFFFFFFFLL) return fail(ctx, PCV_ERR_INVALID_ARG, "iteration counter exceeds 32 bits");
  const int64_t nw = ctx->m.n_warmup;
  if (ctx->m.rhat_mode == PCV_RHAT_SHIFTED_SUMS && nw > 0 && ctx->t < nw && ctx->t + n_iter >= nw) {
    // shifted sums: the fold centres C_k are fixed when the warm-up ends
    const int64_t first = nw - ctx->t;
    TRY(step_run(ctx, first));
    CK(launch_center(ctx->m, ctx->st));
    return step_run(ctx, n_iter - first);
  }
  return step_run(ctx, n_iter);
}

static pcv_status step_run(pcv_ctx ctx, int64_t n_iter) {
  if (ctx->path == PATH_VALU) {
    // one launch runs many whole transitions; chunk to keep launches bounded
    const int64_t chunk = 256;
    for (int64_t done = 0; done < n_iter; done += chunk) {
      const int it = static_cast<int>(std::min<int64_t>(chunk, n_iter - done));
      if (ctx->ev_used + 2 > 4096) timing_collect(ctx);
      timing_begin(ctx);
      CK(launch_valu(ctx->m, ctx->Xv, ctx->fp64, ctx->pb, ctx->W, 0, ctx->t + done, it, 0, ctx->st));
      timing_end(ctx);
    }
    ctx->t += n_iter;
    return PCV_OK;
  }
  const bool use_graph =
      ctx->graphs && !ctx->timing && (ctx->path == PATH_MFMA || ctx->path == PATH_VALU_SPLIT) && n_iter > 0;
  if (use_graph) {
    TRY(capture_transition(ctx));
  }
  if (use_graph && ctx->graph_exec) {
    ctx->t_host = ctx->t;
    CK(hipMemcpyAsync(ctx->m.t_dev, &ctx->t_host, sizeof(int64_t), hipMemcpyHostToDevice, ctx->st));
    for (int64_t i = 0; i < n_iter; ++i) CK(hipGraphLaunch(ctx->graph_exec, ctx->st));
    ctx->t += n_iter;
    // t_host must stay unchanged until the copy above has run
    CK(hipStreamSynchronize(ctx->st));
    return PCV_OK;
  }
  for (int64_t i = 0; i < n_iter; ++i) {
    TRY(transition_split(ctx, ctx->t));
    ctx->t += 1;
  }
  return PCV_OK;
}

static pcv_status run_diag(pcv_ctx ctx, int64_t N, std::vector<double>& fold, double scal[5]) {
  CK(launch_diag(ctx->m, N, ctx->fold_buf, ctx->dscal, ctx->st));
  fold.resize(6 * static_cast<size_t>(ctx->m.KP));
  CK(hipMemcpyAsync(fold.data(), ctx->fold_buf, sizeof(double) * fold.size(), hipMemcpyDeviceToHost, ctx->st));
  CK(hipMemcpyAsync(scal, ctx->dscal, sizeof(double) * 5, hipMemcpyDeviceToHost, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  return PCV_OK;
}

pcv_status pcv_diagnostics(pcv_ctx ctx, pcv_diag* out) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!out) return fail(ctx, PCV_ERR_INVALID_ARG, "null output");
  const int64_t N = std::max<int64_t>(0, ctx->t - ctx->m.n_warmup);
  out->n_iter = ctx->t;
  out->n_draws = N;
  if (N < 2) return fail(ctx, PCV_ERR_STATE, "fewer than 2 post-warm-up draws");
  std::vector<double> fold;
  double scal[5];
  TRY(run_diag(ctx, N, fold, scal));
  const int K = ctx->m.KP;   // posteriors: folds x models
  const double LN = static_cast<double>(ctx->m.L) * N;
  out->elpd = scal[0];
  out->rhat_max = scal[1];
  out->mcse = std::sqrt(scal[2]);
  out->ess = LN * scal[3] / scal[4];
  std::vector<int64_t> na(ctx->m.C), nd(ctx->m.C);
  CK(hipMemcpy(na.data(), ctx->m.nacc, sizeof(int64_t) * na.size(), hipMemcpyDeviceToHost));
  CK(hipMemcpy(nd.data(), ctx->m.ndiv, sizeof(int64_t) * nd.size(), hipMemcpyDeviceToHost));
  int64_t sa = 0, sd = 0;
  for (int64_t c = 0; c < ctx->m.C; ++c) {
    sa += na[c];
    sd += nd[c];
  }
  out->accept_rate = static_cast<double>(sa) / (static_cast<double>(ctx->m.C) * N);
  out->n_divergent = sd;
  if (out->rhat_fold) std::memcpy(out->rhat_fold, fold.data() + K, sizeof(double) * K);
  if (out->ess_fold) std::memcpy(out->ess_fold, fold.data() + 4 * static_cast<size_t>(K), sizeof(double) * K);
  return PCV_OK;
}

pcv_status pcv_elpd(pcv_ctx ctx, double* elpd, double* mcse, double* elpd_fold, double* mcse_fold) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  const int64_t N = std::max<int64_t>(0, ctx->t - ctx->m.n_warmup);
  if (N < 1) return fail(ctx, PCV_ERR_STATE, "no post-warm-up draw");
  std::vector<double> fold;
  double scal[5];
  TRY(run_diag(ctx, N, fold, scal));
  const int K = ctx->m.KP;   // posteriors: folds x models
  if (elpd) *elpd = scal[0];
  if (mcse) *mcse = std::sqrt(scal[2]);
  if (elpd_fold) std::memcpy(elpd_fold, fold.data(), sizeof(double) * K);
  if (mcse_fold)
    for (int k = 0; k < K; ++k) mcse_fold[k] = std::sqrt(fold[5 * static_cast<size_t>(K) + k]);
  return PCV_OK;
}

// Block-shuffle replicates into device buffers rep (KP*R) and mx (R), both
// written in full by the kernels, then to the caller's host arrays.
static pcv_status shuffle_run(pcv_ctx ctx, int64_t N, int32_t R, uint64_t seed, double* rep, double* mx,
                              double* rhat_max_rep, double* rhat_rep) {
  const size_t nrep = static_cast<size_t>(ctx->m.KP) * R;
  hipError_t e = launch_shuffle(ctx->m, N, R, static_cast<uint32_t>(seed & 0xFFFFFFFFu),
                                static_cast<uint32_t>(seed >> 32), rep, mx, ctx->st);
  if (e == hipSuccess) e = hipMemcpyAsync(rhat_max_rep, mx, sizeof(double) * R, hipMemcpyDeviceToHost, ctx->st);
  if (e == hipSuccess && rhat_rep)
    e = hipMemcpyAsync(rhat_rep, rep, sizeof(double) * nrep, hipMemcpyDeviceToHost, ctx->st);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
  if (e != hipSuccess) {
    ctx->dead = true;
    return fail(ctx, PCV_ERR_DEVICE, hipGetErrorString(e));
  }
  return PCV_OK;
}

static pcv_status shuffle_check(pcv_ctx ctx, int32_t R, const double* rhat_max_rep, int64_t* N) {
  if (R < 1 || !rhat_max_rep) return fail(ctx, PCV_ERR_INVALID_ARG, "R >= 1 and an output buffer are required");
  *N = std::max<int64_t>(0, ctx->t - ctx->m.n_warmup);
  if (*N < 2) return fail(ctx, PCV_ERR_STATE, "fewer than 2 post-warm-up draws");
  return PCV_OK;
}

pcv_status pcv_shuffle_benchmark(pcv_ctx ctx, int32_t R, uint64_t seed, double* rhat_max_rep, double* rhat_rep) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  int64_t N = 0;
  TRY(shuffle_check(ctx, R, rhat_max_rep, &N));
  double *rep, *mx;
  const size_t nrep = static_cast<size_t>(ctx->m.KP) * R;
  if (hipMalloc(&rep, sizeof(double) * nrep) != hipSuccess) return fail(ctx, PCV_ERR_NOMEM, "hipMalloc failed");
  if (hipMalloc(&mx, sizeof(double) * R) != hipSuccess) {
    (void)hipFree(rep);
    return fail(ctx, PCV_ERR_NOMEM, "hipMalloc failed");
  }
  const pcv_status s = shuffle_run(ctx, N, R, seed, rep, mx, rhat_max_rep, rhat_rep);
  (void)hipFree(rep);
  (void)hipFree(mx);
  return s;
}

pcv_status pcv_shuffle_benchmark_noalloc(pcv_ctx ctx, int32_t R, uint64_t seed, double* rhat_max_rep,
                                         double* rhat_rep) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  int64_t N = 0;
  TRY(shuffle_check(ctx, R, rhat_max_rep, &N));
  const int64_t need = (static_cast<int64_t>(ctx->m.KP) + 1) * R;
  if (need > PCV_SHUFFLE_NOALLOC_MAX_DOUBLES)
    return fail(ctx, PCV_ERR_INVALID_ARG,
                "(K + 1) * R = " + std::to_string(need) + " doubles exceed the static scratch of " +
                    std::to_string(PCV_SHUFFLE_NOALLOC_MAX_DOUBLES) + " (use pcv_shuffle_benchmark)");
  if (!ctx->noalloc_scratch) return fail(ctx, PCV_ERR_STATE, "the scratch array of this device was not resolved");
  double* rep = ctx->noalloc_scratch;
  double* mx = rep + static_cast<int64_t>(ctx->m.KP) * R;
  return shuffle_run(ctx, N, R, seed, rep, mx, rhat_max_rep, rhat_rep);
}

pcv_status pcv_logdensity_grad(pcv_ctx ctx, const double* theta_dev, double* logp_dev, double* grad_dev,
                               int32_t want_grad) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!theta_dev || !logp_dev || (want_grad && !grad_dev)) return fail(ctx, PCV_ERR_INVALID_ARG, "null pointer");
  DevModel& m = ctx->m;
  CK(launch_to_dc(theta_dev, m.q1, m.C, m.d, ctx->st));
  TRY(eval_q1(ctx));
  CK(hipMemcpyAsync(logp_dev, m.logp1, sizeof(double) * m.C, hipMemcpyDeviceToDevice, ctx->st));
  if (want_grad) CK(launch_to_cd(m.g1, grad_dev, m.C, m.d, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  return PCV_OK;
}

pcv_status pcv_leapfrog(pcv_ctx ctx, const double* q_dev, const double* p_dev, int32_t n_steps, double* q_out_dev,
                        double* p_out_dev, double* logp_out_dev, double* grad_out_dev) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!q_dev || !p_dev || !q_out_dev || !p_out_dev || !logp_out_dev || !grad_out_dev || n_steps < 1)
    return fail(ctx, PCV_ERR_INVALID_ARG, "null pointer or n_steps < 1");
  DevModel& m = ctx->m;
  CK(launch_to_dc(q_dev, m.q1, m.C, m.d, ctx->st));
  CK(launch_to_dc(p_dev, m.pm, m.C, m.d, ctx->st));
  if (ctx->path == PATH_VALU) {
    CK(launch_valu(m, ctx->Xv, ctx->fp64, ctx->pb, ctx->W, 2, 0, 0, n_steps, ctx->st));
  } else {
    TRY(split_partials(ctx, false));
    TRY(split_reduce(ctx, 0));
    CK(launch_kick_drift(m, ctx->st));
    for (int s = 0; s < n_steps; ++s) {
      const bool last = s == n_steps - 1;
      TRY(split_partials(ctx, last));
      TRY(split_reduce(ctx, last ? 2 : 1));
    }
    CK(launch_value_finish(m, ctx->Vpart, split_count(ctx), ctx->st));
  }
  CK(launch_to_cd(m.q1, q_out_dev, m.C, m.d, ctx->st));
  CK(launch_to_cd(m.pm, p_out_dev, m.C, m.d, ctx->st));
  CK(launch_to_cd(m.g1, grad_out_dev, m.C, m.d, ctx->st));
  CK(hipMemcpyAsync(logp_out_dev, m.logp1, sizeof(double) * m.C, hipMemcpyDeviceToDevice, ctx->st));
  CK(hipStreamSynchronize(ctx->st));
  return PCV_OK;
}

pcv_status pcv_get_state(pcv_ctx ctx, double* theta, double* logp, double* s) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  DevModel& m = ctx->m;
  CK(hipStreamSynchronize(ctx->st));
  if (theta) {
    std::vector<double> dc(static_cast<size_t>(m.d) * m.C);
    CK(hipMemcpy(dc.data(), m.q0, sizeof(double) * dc.size(), hipMemcpyDeviceToHost));
    for (int64_t c = 0; c < m.C; ++c)
      for (int64_t j = 0; j < m.d; ++j) theta[c * m.d + j] = dc[j * m.C + c];
  }
  if (logp) CK(hipMemcpy(logp, m.logp0, sizeof(double) * m.C, hipMemcpyDeviceToHost));
  if (s) CK(hipMemcpy(s, m.s0, sizeof(double) * m.C, hipMemcpyDeviceToHost));
  return PCV_OK;
}

pcv_status pcv_set_state(pcv_ctx ctx, const double* theta) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  DevModel& m = ctx->m;
  if (!theta || !finite_all(theta, m.C * m.d)) return fail(ctx, PCV_ERR_INVALID_ARG, "theta must be finite");
  std::vector<double> dc(static_cast<size_t>(m.d) * m.C);
  for (int64_t c = 0; c < m.C; ++c)
    for (int64_t j = 0; j < m.d; ++j) dc[j * m.C + c] = theta[c * m.d + j];
  CK(hipStreamSynchronize(ctx->st));
  CK(hipMemcpy(m.q1, dc.data(), sizeof(double) * dc.size(), hipMemcpyHostToDevice));
  TRY(eval_q1(ctx));
  TRY(adopt_q1(ctx));
  CK(hipStreamSynchronize(ctx->st));
  return PCV_OK;
}

pcv_status pcv_get_accumulators(pcv_ctx ctx, double* Z, double* U, double* U2, double* V, double* V2,
                                double* blk_mean, double* blk_m2, int64_t* n_accept, int64_t* n_divergent) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  DevModel& m = ctx->m;
  CK(hipStreamSynchronize(ctx->st));
  const size_t C = m.C, DC = static_cast<size_t>(m.D) * m.C;
  if (Z) CK(hipMemcpy(Z, m.Z, sizeof(double) * C, hipMemcpyDeviceToHost));
  if (U) CK(hipMemcpy(U, m.U, sizeof(double) * C, hipMemcpyDeviceToHost));
  if (U2) CK(hipMemcpy(U2, m.U2, sizeof(double) * C, hipMemcpyDeviceToHost));
  if (V) CK(hipMemcpy(V, m.V, sizeof(double) * C, hipMemcpyDeviceToHost));
  if (V2) CK(hipMemcpy(V2, m.V2, sizeof(double) * C, hipMemcpyDeviceToHost));
  if (blk_mean) CK(hipMemcpy(blk_mean, m.bmean, sizeof(double) * DC, hipMemcpyDeviceToHost));
  if (blk_m2) CK(hipMemcpy(blk_m2, m.bm2, sizeof(double) * DC, hipMemcpyDeviceToHost));
  if (n_accept) CK(hipMemcpy(n_accept, m.nacc, sizeof(int64_t) * C, hipMemcpyDeviceToHost));
  if (n_divergent) CK(hipMemcpy(n_divergent, m.ndiv, sizeof(int64_t) * C, hipMemcpyDeviceToHost));
  return PCV_OK;
}

// ---- checkpoints ---------------------------------------------------------

}  // extern "C"

namespace {

struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t family, precision, fold_kind;
  int64_t n, p, d, C;
  int32_t K, L, D, b, Gb, S, rhat_mode, scores;
  int64_t draws_cap;
  uint64_t seed;
  int64_t chain_offset, n_warmup;
  double eps;
  uint64_t fingerprint;
  int64_t t;
  uint64_t payload_bytes;
  uint64_t payload_hash;
};
static_assert(sizeof(CkptHeader) == 160, "checkpoint header has no padding");
constexpr char kCkptMagic[8] = {'P', 'C', 'V', 'C', 'K', 'P', 'T', '2'};

CkptHeader ckpt_header_of(pcv_ctx ctx) {
  const DevModel& m = ctx->m;
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = 2;
  h.family = m.family;
  h.precision = ctx->prec;
  h.fold_kind = m.fold_kind;
  h.n = m.n;
  h.p = m.p;
  h.d = m.d;
  h.C = m.C;
  h.K = m.K;
  h.L = m.L;
  h.D = m.D;
  h.b = m.b;
  h.Gb = m.Gb;
  h.S = m.S;
  h.rhat_mode = m.rhat_mode;
  h.scores = m.scores;
  h.draws_cap = m.draws_cap;
  h.seed = (static_cast<uint64_t>(m.key1) << 32) | m.key0;
  h.chain_offset = m.chain_offset;
  h.n_warmup = m.n_warmup;
  h.eps = m.eps;
  h.fingerprint = ctx->fingerprint;
  return h;
}

// The device arrays a checkpoint holds, in file order: the accepted state and
// every online accumulator.
struct CkptArray {
  void* dev;
  size_t bytes;
};
std::vector<CkptArray> ckpt_arrays(pcv_ctx ctx) {
  const DevModel& m = ctx->m;
  const size_t C = m.C, dC = static_cast<size_t>(m.d) * m.C, DC = static_cast<size_t>(m.D) * m.C;
  const size_t K = static_cast<size_t>(m.KP);
  // the inverse mass is sampler state (pcv_adapt rewrites it); the step size
  // travels in the header
  std::vector<CkptArray> a = {{m.q0, 8 * dC},  {m.g0, 8 * dC},  {m.logp0, 8 * C}, {m.s0, 8 * C},
                              {m.Z, 8 * C},    {m.U, 8 * C},    {m.U2, 8 * C},    {m.V, 8 * C},
                              {m.V2, 8 * C},   {m.bmean, 8 * DC}, {m.bm2, 8 * DC}, {m.nacc, 8 * C},
                              {m.ndiv, 8 * C}, {m.wsum, 8 * C}, {m.center, 8 * K},
                              {const_cast<double*>(m.minv), 8 * static_cast<size_t>(m.d)}};
  const size_t Lnnz = static_cast<size_t>(m.L) * ctx->test_ptr_host[m.K];
  if (m.hs1) a.push_back({m.hs1, 8 * C});
  if (m.hs2) a.push_back({m.hs2, 8 * Lnnz});
  if (m.dx) a.push_back({m.dx, 8 * Lnnz});
  if (m.dxx) a.push_back({m.dxx, 8 * static_cast<size_t>(m.L) * ctx->sq_ptr_host[m.K]});
  if (m.draws) a.push_back({m.draws, 8 * static_cast<size_t>(m.draws_cap) * C});
  return a;
}

}  // namespace

extern "C" {

pcv_status pcv_save(pcv_ctx ctx, const char* path) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!path || !*path) return fail(ctx, PCV_ERR_INVALID_ARG, "null path");
  CK(hipStreamSynchronize(ctx->st));
  const std::vector<CkptArray> arrs = ckpt_arrays(ctx);
  size_t total = 0;
  for (const CkptArray& a : arrs) total += a.bytes;
  std::vector<unsigned char> payload(total);
  size_t off = 0;
  for (const CkptArray& a : arrs) {
    CK(hipMemcpy(payload.data() + off, a.dev, a.bytes, hipMemcpyDeviceToHost));
    off += a.bytes;
  }
  CkptHeader h = ckpt_header_of(ctx);
  h.t = ctx->t;
  h.payload_bytes = total;
  h.payload_hash = fp_mix(0xcbf29ce484222325ULL, payload.data(), total);
  // write to a temporary name, then rename: a crash never leaves a torn file
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(ctx, PCV_ERR_INVALID_ARG, "cannot open " + tmp + " for writing");
  const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(payload.data(), 1, total, f) == total;
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed) {
    std::remove(tmp.c_str());
    return fail(ctx, PCV_ERR_INVALID_ARG, "write to " + tmp + " failed");
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(ctx, PCV_ERR_INVALID_ARG, std::string("cannot rename checkpoint to ") + path);
  }
  return PCV_OK;
}

pcv_status pcv_load(pcv_ctx ctx, const char* path) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!path || !*path) return fail(ctx, PCV_ERR_INVALID_ARG, "null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(ctx, PCV_ERR_INVALID_ARG, std::string("cannot open ") + path);
  CkptHeader h{};
  const bool got = std::fread(&h, sizeof(h), 1, f) == 1;
  const std::vector<CkptArray> arrs = ckpt_arrays(ctx);
  size_t total = 0;
  for (const CkptArray& a : arrs) total += a.bytes;
  std::vector<unsigned char> payload;
  bool body = false;
  if (got && std::memcmp(h.magic, kCkptMagic, 8) == 0 && h.payload_bytes == total) {
    payload.resize(total);
    body = std::fread(payload.data(), 1, total, f) == total && std::fgetc(f) == EOF;
  }
  std::fclose(f);
  if (!got || std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 2)
    return fail(ctx, PCV_ERR_INVALID_ARG, "not a checkpoint of this library");
  CkptHeader want = ckpt_header_of(ctx);
  want.t = h.t;
  want.eps = h.eps;   // tuning state, restored below
  want.payload_bytes = h.payload_bytes;
  want.payload_hash = h.payload_hash;
  if (std::memcmp(&want, &h, sizeof(h)) != 0)
    return fail(ctx, PCV_ERR_INVALID_ARG, "checkpoint is of another model, data, fold set or precision");
  if (!body || fp_mix(0xcbf29ce484222325ULL, payload.data(), total) != h.payload_hash)
    return fail(ctx, PCV_ERR_INVALID_ARG, "checkpoint is truncated or corrupted");
  if (h.t < 0 || h.t > 0xFFFFFFFFLL) return fail(ctx, PCV_ERR_INVALID_ARG, "checkpoint iteration out of range");
  if (!(h.eps > 0) || !std::isfinite(h.eps)) return fail(ctx, PCV_ERR_INVALID_ARG, "checkpoint step size invalid");
  {
    // the inverse mass sits last in the payload: it must be positive
    const size_t off_minv = total - 8 * static_cast<size_t>(ctx->m.d);
    for (int64_t j = 0; j < ctx->m.d; ++j) {
      double v;
      std::memcpy(&v, payload.data() + off_minv + 8 * j, 8);
      if (!(v > 0) || !std::isfinite(v)) return fail(ctx, PCV_ERR_INVALID_ARG, "checkpoint inverse mass invalid");
    }
  }
  CK(hipStreamSynchronize(ctx->st));
  size_t off = 0;
  for (const CkptArray& a : arrs) {
    CK(hipMemcpy(a.dev, payload.data() + off, a.bytes, hipMemcpyHostToDevice));
    off += a.bytes;
  }
  ctx->t = h.t;
  if (h.eps != ctx->m.eps) {
    ctx->m.eps = h.eps;
    drop_graph(ctx);   // a captured transition holds the old step size
  }
  return PCV_OK;
}

// ---- Hyvaerinen and Dawid-Sebastiani scores ---------------------------------

}  // extern "C"

namespace {

// log|S| and m' S^-1 m by Cholesky (S symmetric, n x n, overwritten); false if
// S is not positive definite.
bool chol_logdet_quad(std::vector<double>& S, int n, std::vector<double> m, double* logdet, double* quad) {
  for (int j = 0; j < n; ++j) {
    double d = S[static_cast<size_t>(j) * n + j];
    for (int k = 0; k < j; ++k) d -= S[static_cast<size_t>(j) * n + k] * S[static_cast<size_t>(j) * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    S[static_cast<size_t>(j) * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double e = S[static_cast<size_t>(i) * n + j];
      for (int k = 0; k < j; ++k) e -= S[static_cast<size_t>(i) * n + k] * S[static_cast<size_t>(j) * n + k];
      S[static_cast<size_t>(i) * n + j] = e / d;
    }
  }
  double ld = 0.0, q = 0.0;
  for (int i = 0; i < n; ++i) {   // forward solve L z = m, q = |z|^2
    double e = m[i];
    for (int k = 0; k < i; ++k) e -= S[static_cast<size_t>(i) * n + k] * m[k];
    m[i] = e / S[static_cast<size_t>(i) * n + i];
    q += m[i] * m[i];
    ld += 2.0 * std::log(S[static_cast<size_t>(i) * n + i]);
  }
  *logdet = ld;
  *quad = q;
  return true;
}

}  // namespace

extern "C" {

pcv_status pcv_scores(pcv_ctx ctx, double* hs, double* hs_fold, double* dss, double* dss_fold) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  const DevModel& m = ctx->m;
  if (((hs || hs_fold) && !(m.scores & PCV_SCORE_HS)) || ((dss || dss_fold) && !(m.scores & PCV_SCORE_DSS)))
    return fail(ctx, PCV_ERR_INVALID_ARG, "a requested score was not enabled in pcv_model.scores");
  const int64_t N = std::max<int64_t>(0, ctx->t - m.n_warmup);
  const int K = m.K, L = m.L;
  const double LN = static_cast<double>(L) * N;
  if (N < 2) return fail(ctx, PCV_ERR_STATE, "scores need at least 2 post-warm-up draws");
  CK(hipStreamSynchronize(ctx->st));
  const std::vector<int32_t>& tp = ctx->test_ptr_host;
  const size_t Lnnz = static_cast<size_t>(L) * tp[K];
  if (m.scores & PCV_SCORE_HS) {
    std::vector<double> h1(m.C), h2(Lnnz);
    CK(hipMemcpy(h1.data(), m.hs1, 8 * h1.size(), hipMemcpyDeviceToHost));
    CK(hipMemcpy(h2.data(), m.hs2, 8 * h2.size(), hipMemcpyDeviceToHost));
    double tot = 0.0;
    for (int k = 0; k < K; ++k) {
      const int v = tp[k + 1] - tp[k];
      double s1 = 0.0, sq = 0.0;
      for (int l = 0; l < L; ++l) s1 += h1[static_cast<size_t>(k) * L + l];
      for (int a = 0; a < v; ++a) {
        double s2 = 0.0;
        for (int l = 0; l < L; ++l) s2 += h2[static_cast<size_t>(L) * tp[k] + static_cast<size_t>(l) * v + a];
        const double mu2 = s2 / LN;
        sq += mu2 * mu2;
      }
      const double hk = -2.0 * s1 / LN + sq;
      if (hs_fold) hs_fold[k] = hk;
      tot += hk;
    }
    if (hs) *hs = tot;
  }
  if (m.scores & PCV_SCORE_DSS) {
    const std::vector<int64_t>& sp = ctx->sq_ptr_host;
    std::vector<double> x(Lnnz), xx(static_cast<size_t>(L) * sp[K]);
    CK(hipMemcpy(x.data(), m.dx, 8 * x.size(), hipMemcpyDeviceToHost));
    CK(hipMemcpy(xx.data(), m.dxx, 8 * xx.size(), hipMemcpyDeviceToHost));
    double tot = 0.0;
    for (int k = 0; k < K; ++k) {
      const int v = tp[k + 1] - tp[k];
      std::vector<double> sx(v, 0.0), S(static_cast<size_t>(v) * v, 0.0);
      for (int l = 0; l < L; ++l) {
        for (int a = 0; a < v; ++a) sx[a] += x[static_cast<size_t>(L) * tp[k] + static_cast<size_t>(l) * v + a];
        const size_t o2 = static_cast<size_t>(L) * sp[k] + static_cast<size_t>(l) * v * v;
        for (size_t ab = 0; ab < static_cast<size_t>(v) * v; ++ab) S[ab] += xx[o2 + ab];
      }
      std::vector<double> mv(v);
      for (int a = 0; a < v; ++a) mv[a] = sx[a] / LN;
      for (int a = 0; a < v; ++a)
        for (int b = 0; b < v; ++b)
          S[static_cast<size_t>(a) * v + b] = (S[static_cast<size_t>(a) * v + b] - sx[a] * sx[b] / LN) / (LN - 1.0);
      double ld = 0.0, q = 0.0;
      const double dk = chol_logdet_quad(S, v, mv, &ld, &q) ? -ld - q : NAN;
      if (dss_fold) dss_fold[k] = dk;
      tot += dk;
    }
    if (dss) *dss = tot;
  }
  return PCV_OK;
}

// ---- stored draws (Algorithm 1) and post-hoc diagnostics ----------------------

static int64_t stored_draws(pcv_ctx ctx) {
  return std::min<int64_t>(std::max<int64_t>(0, ctx->t - ctx->m.n_warmup), ctx->m.draws_cap);
}

pcv_status pcv_get_draws(pcv_ctx ctx, double* s, int64_t n_max, int64_t* n_out) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!ctx->m.draws) return fail(ctx, PCV_ERR_INVALID_ARG, "draws are not stored (pcv_model.store_draws = 0)");
  if (n_max < 0 || (n_max > 0 && !s)) return fail(ctx, PCV_ERR_INVALID_ARG, "bad output buffer");
  const int64_t n = std::min(stored_draws(ctx), n_max), C = ctx->m.C;
  CK(hipStreamSynchronize(ctx->st));
  std::vector<double> buf(static_cast<size_t>(n) * C);
  if (n > 0) CK(hipMemcpy(buf.data(), ctx->m.draws, 8 * buf.size(), hipMemcpyDeviceToHost));
  for (int64_t c = 0; c < C; ++c)
    for (int64_t i = 0; i < n; ++i) s[c * n + i] = buf[static_cast<size_t>(i) * C + c];
  if (n_out) *n_out = n;
  return PCV_OK;
}

pcv_status pcv_posthoc(pcv_ctx ctx, pcv_posthoc_diag* out) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!out) return fail(ctx, PCV_ERR_INVALID_ARG, "null output");
  if (!ctx->m.draws) return fail(ctx, PCV_ERR_INVALID_ARG, "draws are not stored (pcv_model.store_draws = 0)");
  const int64_t N = stored_draws(ctx), C = ctx->m.C;
  const int K = ctx->m.KP, L = ctx->m.L;   // posteriors: folds x models
  if (N < 4) return fail(ctx, PCV_ERR_STATE, "post-hoc diagnostics need at least 4 stored draws");
  std::vector<double> s(static_cast<size_t>(N) * C);
  int64_t got = 0;
  TRY(pcv_get_draws(ctx, s.data(), N, &got));
  double elpd = 0.0, var = 0.0, s2 = 0.0, sig2 = 0.0;
  out->rhat_max = out->split_rhat_max = out->rank_rhat_max = -INFINITY;
  for (int k = 0; k < K; ++k) {
    PosthocFold f{};
    posthoc_fold(s.data() + static_cast<size_t>(k) * L * N, L, N, ctx->m.b, f);
    elpd += f.log_fhat;
    var += f.sig2rel / (static_cast<double>(L) * N);
    s2 += f.s2rel;
    sig2 += f.sig2rel;
    out->rhat_max = std::max(out->rhat_max, f.rhat);
    out->split_rhat_max = std::max(out->split_rhat_max, f.split_rhat);
    out->rank_rhat_max = std::max(out->rank_rhat_max, f.rank_rhat);
    if (out->rhat_fold) out->rhat_fold[k] = f.rhat;
    if (out->split_rhat_fold) out->split_rhat_fold[k] = f.split_rhat;
    if (out->rank_rhat_fold) out->rank_rhat_fold[k] = f.rank_rhat;
  }
  out->elpd = elpd;
  out->mcse = std::sqrt(var);
  out->ess = static_cast<double>(L) * N * s2 / sig2;
  out->n_draws = N;
  return PCV_OK;
}

// ---- model comparison --------------------------------------------------------

}  // extern "C"

namespace {

// Sections 2.3 and 4.1 over per-fold estimates of two models on the same K
// folds: Delta and its fold variance (eqs sel-cv, norm-approx), and the
// Monte Carlo error from both models' fold variances (eq mc-var).
void compare_folds(const std::vector<double>& ea, const std::vector<double>& ma, const std::vector<double>& eb,
                   const std::vector<double>& mb, int K, pcv_comparison* out) {
  double delta = 0.0, var_mc = 0.0;
  for (int k = 0; k < K; ++k) {
    delta += ea[k] - eb[k];
    var_mc += ma[k] * ma[k] + mb[k] * mb[k];
  }
  double ss = 0.0;
  for (int k = 0; k < K; ++k) {
    const double e = (ea[k] - eb[k]) - delta / K;
    ss += e * e;
  }
  const double sigma2 = K > 1 ? ss / (K - 1) : NAN;
  double prob;
  if (sigma2 > 0.0) prob = 0.5 * std::erfc(-delta / std::sqrt(2.0 * K * sigma2));
  else prob = delta == 0.0 ? 0.5 : (delta > 0.0 ? 1.0 : 0.0);
  out->delta = delta;
  out->sigma2 = sigma2;
  out->prob_a_better = prob;
  out->mcse = std::sqrt(var_mc);
  if (out->delta_fold)
    for (int k = 0; k < K; ++k) out->delta_fold[k] = ea[k] - eb[k];
}

}  // namespace

extern "C" {

pcv_status pcv_compare(pcv_ctx a, pcv_ctx b, pcv_comparison* out) {
  if (!usable(a) || !usable(b)) return PCV_ERR_STATE;
  if (!out) return fail(a, PCV_ERR_INVALID_ARG, "null output");
  if (a->m.M > 1 || b->m.M > 1)
    return fail(a, PCV_ERR_INVALID_ARG, "runs with several models: use pcv_compare_models");
  if (a->m.K != b->m.K || a->fold_fp != b->fold_fp)
    return fail(a, PCV_ERR_INVALID_ARG, "the two models were not evaluated on the same folds");
  const int K = a->m.K;
  std::vector<double> ea(K), ma(K), eb(K), mb(K);
  double ta = 0.0, sa = 0.0, tb = 0.0, sb = 0.0;
  pcv_status st = pcv_elpd(a, &ta, &sa, ea.data(), ma.data());
  if (st != PCV_OK) return st;
  st = pcv_elpd(b, &tb, &sb, eb.data(), mb.data());
  if (st != PCV_OK) return fail(a, st, std::string("model B: ") + b->err);
  compare_folds(ea, ma, eb, mb, K, out);
  return PCV_OK;
}

pcv_status pcv_elpd_model(pcv_ctx ctx, int32_t model, double* elpd, double* mcse, double* elpd_fold,
                          double* mcse_fold) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (model < 0 || model >= ctx->m.M) return fail(ctx, PCV_ERR_INVALID_ARG, "model index out of range");
  const int K = ctx->m.K, KP = ctx->m.KP;
  std::vector<double> ef(KP), mf(KP);
  TRY(pcv_elpd(ctx, nullptr, nullptr, ef.data(), mf.data()));
  double e = 0.0, v = 0.0;
  for (int k = 0; k < K; ++k) {
    const double mk = mf[static_cast<size_t>(model) * K + k];
    e += ef[static_cast<size_t>(model) * K + k];
    v += mk * mk;
    if (elpd_fold) elpd_fold[k] = ef[static_cast<size_t>(model) * K + k];
    if (mcse_fold) mcse_fold[k] = mk;
  }
  if (elpd) *elpd = e;
  if (mcse) *mcse = std::sqrt(v);
  return PCV_OK;
}

pcv_status pcv_compare_models(pcv_ctx ctx, int32_t a, int32_t b, pcv_comparison* out) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!out) return fail(ctx, PCV_ERR_INVALID_ARG, "null output");
  if (a < 0 || a >= ctx->m.M || b < 0 || b >= ctx->m.M) return fail(ctx, PCV_ERR_INVALID_ARG, "model index out of range");
  const int K = ctx->m.K;
  std::vector<double> ea(K), ma(K), eb(K), mb(K);
  TRY(pcv_elpd_model(ctx, a, nullptr, nullptr, ea.data(), ma.data()));
  TRY(pcv_elpd_model(ctx, b, nullptr, nullptr, eb.data(), mb.data()));
  compare_folds(ea, ma, eb, mb, K, out);
  return PCV_OK;
}

// ---- autotuning ------------------------------------------------------------

}  // extern "C"

namespace {

std::string tune_key(pcv_ctx ctx) {
  const DevModel& m = ctx->m;
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  char buf[512];
  const char* path = ctx->path == PATH_MFMA ? "mfma" : ctx->path == PATH_VALU_SPLIT ? "valu-split" : "valu";
  std::snprintf(buf, sizeof buf, "%s fam=%d prec=%d folds=%d n=%lld p=%lld C=%lld K=%d L=%d groups=%d arch=%s",
                path, m.family, ctx->prec, m.fold_kind,
                static_cast<long long>(m.n), static_cast<long long>(m.p), static_cast<long long>(m.C), m.K, m.L,
                m.n_groups, arch.c_str());
  return buf;
}

// The cache is a flat JSON object, one entry per line:
//   "<key>": {"cfg": <int>, "ms": <float>},
struct TuneEntry {
  std::string key;
  int cfg;
  double ms;
};

std::vector<TuneEntry> cache_read(const char* path) {
  std::vector<TuneEntry> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[2048];
  while (std::fgets(line, sizeof line, f)) {
    const char* q1 = std::strchr(line, '"');
    if (!q1) continue;
    const char* q2 = std::strchr(q1 + 1, '"');
    if (!q2) continue;
    const char* c = std::strstr(q2, "\"cfg\":");
    const char* t = std::strstr(q2, "\"ms\":");
    TuneEntry e{std::string(q1 + 1, q2), 0, 0.0};
    if (c && t && std::sscanf(c + 6, "%d", &e.cfg) == 1 && std::sscanf(t + 5, "%lf", &e.ms) == 1) out.push_back(e);
  }
  std::fclose(f);
  return out;
}

bool cache_write(const char* path, const std::vector<TuneEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = std::fprintf(f, "{\n") > 0;
  for (size_t i = 0; i < entries.size(); ++i)
    ok = ok && std::fprintf(f, "  \"%s\": {\"cfg\": %d, \"ms\": %.9g}%s\n", entries[i].key.c_str(), entries[i].cfg,
                            entries[i].ms, i + 1 < entries.size() ? "," : "") > 0;
  ok = ok && std::fprintf(f, "}\n") > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

void drop_graph(pcv_ctx ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
}

// MFMA path: ns row splits per chain tile (the partial buffers grow if needed).
pcv_status apply_splits(pcv_ctx ctx, int ns) {
  const int tps = (ctx->n_tiles + ns - 1) / ns;
  const int nsp = (ctx->n_tiles + tps - 1) / tps;
  if (nsp > ctx->split_cap) {
    float* g;
    double* v;
    TRY(dalloc(ctx, &g, static_cast<size_t>(nsp) * ctx->m.p * ctx->m.C));
    TRY(dalloc(ctx, &v, static_cast<size_t>(nsp) * ctx->m.C));
    ctx->Gpart = g;
    ctx->Vpart = v;
    ctx->split_cap = nsp;
  }
  ctx->tiles_per_split = tps;
  ctx->n_splits = nsp;
  drop_graph(ctx);
  return PCV_OK;
}

// MFMA launch shape as one autotuner config: MFMA_CFG_SHAPE * shape + splits.
constexpr int MFMA_CFG_SHAPE = 256;
bool mfma_cfg_ok(pcv_ctx ctx, int cfg) {
  const int shape = cfg / MFMA_CFG_SHAPE, ns = cfg % MFMA_CFG_SHAPE;
  return cfg >= 0 && mfma_shape_ok(shape, ctx->m.p) && ns >= 1 &&
         ns <= std::min(64, ctx->n_tiles);
}
pcv_status apply_mfma_cfg(pcv_ctx ctx, int cfg) {
  if (!mfma_cfg_ok(ctx, cfg)) return fail(ctx, PCV_ERR_INVALID_ARG, "invalid MFMA launch configuration");
  TRY(apply_mfma_shape(ctx, cfg / MFMA_CFG_SHAPE));
  return apply_splits(ctx, cfg % MFMA_CFG_SHAPE);
}

bool waves_ok(pcv_ctx ctx, int W) {
  return W >= 1 && W <= 8 && !(ctx->pb >= 32 && W > 4) && ctx->m.n / W >= 8 &&
         valu_smem_bytes(ctx->fp64, W, ctx->m.family, ctx->m.n_groups, ctx->pb) <= 65536;
}

// VALU path: W waves per workgroup, each owning a range of rows.
pcv_status apply_waves(pcv_ctx ctx, int W) {
  const std::vector<int32_t> wr = valu_partition(ctx->m.n, W);
  CK(hipMemcpy(ctx->wave_rows, wr.data(), sizeof(int32_t) * wr.size(), hipMemcpyHostToDevice));
  ctx->W = W;
  return PCV_OK;
}

// Mean time of one gradient evaluation at q1 (a copy of the chain positions;
// q1 and g1 are per-trajectory scratch, so the chains are untouched): the
// fused kernel's gradient launch, or on the split paths the partials launch
// plus the reduction of its partials.
pcv_status time_hot(pcv_ctx ctx, int reps, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  auto launch = [&]() -> pcv_status {
    if (ctx->path == PATH_VALU) {
      CK(launch_valu(ctx->m, ctx->Xv, ctx->fp64, ctx->pb, ctx->W, 1, 0, 0, 0, ctx->st));
      return PCV_OK;
    }
    TRY(split_partials(ctx, false));
    // the split count also sets the reduction's work, so the reduction
    // (mode 0: gradient into the scratch g1) is timed with the partials
    TRY(split_reduce(ctx, 0));
    return PCV_OK;
  };
  pcv_status s = launch();
  if (s == PCV_OK && hipEventRecord(a, ctx->st) != hipSuccess) s = PCV_ERR_DEVICE;
  for (int r = 0; r < reps && s == PCV_OK; ++r) s = launch();
  if (s == PCV_OK && hipEventRecord(b, ctx->st) != hipSuccess) s = PCV_ERR_DEVICE;
  if (s == PCV_OK && hipEventSynchronize(b) != hipSuccess) s = PCV_ERR_DEVICE;
  float t = 0.f;
  if (s == PCV_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) s = PCV_ERR_DEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s != PCV_OK) return fail(ctx, PCV_ERR_DEVICE, "autotune timing failed");
  *ms = static_cast<double>(t) / reps;
  return PCV_OK;
}

}  // namespace

extern "C" {

pcv_status pcv_autotune(pcv_ctx ctx, const char* cache_path, int32_t* config, double* ms) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (ctx->path == PATH_UNFUSED) return fail(ctx, PCV_ERR_UNSUPPORTED, "the plain fp64 path has nothing to tune");
  const std::string key = tune_key(ctx);
  std::vector<TuneEntry> cache = cache_path ? cache_read(cache_path) : std::vector<TuneEntry>{};
  for (const TuneEntry& e : cache) {
    if (e.key != key) continue;
    const bool valid = ctx->path == PATH_MFMA        ? mfma_cfg_ok(ctx, e.cfg)
                       : ctx->path == PATH_VALU_SPLIT ? valu_split_cfg_ok(ctx, e.cfg)
                                                      : waves_ok(ctx, e.cfg);
    if (!valid) break;   // stale entry: tune again
    if (ctx->path == PATH_MFMA) TRY(apply_mfma_cfg(ctx, e.cfg));
    else if (ctx->path == PATH_VALU_SPLIT) TRY(apply_valu_split_cfg(ctx, e.cfg));
    else TRY(apply_waves(ctx, e.cfg));
    if (config) *config = e.cfg;
    if (ms) *ms = e.ms;
    return PCV_OK;
  }
  std::vector<int> cand;
  if (ctx->path == PATH_VALU_SPLIT) {
    // waves per workgroup (2, 4 or 8) and split counts around the analytic
    // choice, scaled to keep the rows per wave: config = VALU_CFG_WAVES * W + splits
    const int ns0 = ctx->n_splits, W0 = ctx->W;
    for (int W : {2, 4, 8})
      for (int f : {2, 3, 4, 6, 8}) {   // ns0 x f / 4
        const int ns = std::max(1, ns0 * f * W0 / (4 * W));
        const int cfg = VALU_CFG_WAVES * W + ns;
        if (valu_split_cfg_ok(ctx, cfg) && std::find(cand.begin(), cand.end(), cfg) == cand.end()) cand.push_back(cfg);
      }
  } else if (ctx->path == PATH_MFMA) {
    // every MFMA launch shape the width allows, each with row-split counts
    // around the analytic choice: config = MFMA_CFG_SHAPE * shape + splits
    const int ns0 = ctx->n_splits, hi = std::min(64, ctx->n_tiles);
    for (int shape : {MFMA_SHAPE_32X32X16, MFMA_SHAPE_32X32X16_IL, MFMA_SHAPE_16X16X32, MFMA_SHAPE_16X16X32_C16})
      for (int ns : {ns0 / 2, ns0 - 2, ns0 - 1, ns0, ns0 + 1, ns0 + 2, 2 * ns0}) {
        if (ns < 1 || ns > hi || !mfma_shape_ok(shape, ctx->m.p)) continue;
        const int tps = (ctx->n_tiles + ns - 1) / ns;
        const int nsp = (ctx->n_tiles + tps - 1) / tps;
        const int cfg = MFMA_CFG_SHAPE * shape + nsp;
        if (std::find(cand.begin(), cand.end(), cfg) == cand.end()) cand.push_back(cfg);
      }
  } else {
    for (int W : {1, 2, 4, 8})
      if (waves_ok(ctx, W)) cand.push_back(W);
  }
  const bool timing = ctx->timing;
  ctx->timing = false;
  CK(hipMemcpyAsync(ctx->m.q1, ctx->m.q0, sizeof(double) * ctx->m.d * ctx->m.C, hipMemcpyDeviceToDevice,
                    ctx->st));
  // two interleaved passes over the candidates, each kept at its faster
  // pass, so that a clock or cache transient does not decide the choice
  const int reps = ctx->path == PATH_MFMA ? 3 : 5;
  std::vector<double> tmin(cand.size(), 0.0);
  pcv_status s = PCV_OK;
  for (int pass = 0; pass < 2 && s == PCV_OK; ++pass) {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const int c = cand[ci];
      s = ctx->path == PATH_MFMA ? apply_mfma_cfg(ctx, c) : ctx->path == PATH_VALU ? apply_waves(ctx, c)
                                                                                   : apply_valu_split_cfg(ctx, c);
      double t = 0.0;
      if (s == PCV_OK) s = time_hot(ctx, reps, &t);
      if (s != PCV_OK) break;
      tmin[ci] = pass == 0 ? t : std::min(tmin[ci], t);
    }
  }
  int best = -1;
  double best_ms = 0.0;
  for (size_t ci = 0; ci < cand.size() && s == PCV_OK; ++ci)
    if (best < 0 || tmin[ci] < best_ms) {
      best = cand[ci];
      best_ms = tmin[ci];
    }
  ctx->timing = timing;
  if (s != PCV_OK) return s;
  TRY(ctx->path == PATH_MFMA   ? apply_mfma_cfg(ctx, best)
      : ctx->path == PATH_VALU ? apply_waves(ctx, best)
                               : apply_valu_split_cfg(ctx, best));
  if (config) *config = best;
  if (ms) *ms = best_ms;
  if (cache_path) {
    bool replaced = false;
    for (TuneEntry& e : cache)
      if (e.key == key) {
        e.cfg = best;
        e.ms = best_ms;
        replaced = true;
      }
    if (!replaced) cache.push_back({key, best, best_ms});
    if (!cache_write(cache_path, cache))
      return fail(ctx, PCV_ERR_INVALID_ARG, std::string("cannot write the tuning cache ") + cache_path);
  }
  return PCV_OK;
}

pcv_status pcv_set_launch_config(pcv_ctx ctx, int32_t config) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (ctx->path == PATH_UNFUSED) return fail(ctx, PCV_ERR_UNSUPPORTED, "the plain fp64 path has no launch shape");
  const bool valid = ctx->path == PATH_MFMA        ? mfma_cfg_ok(ctx, config)
                     : ctx->path == PATH_VALU_SPLIT ? valu_split_cfg_ok(ctx, config)
                                                    : waves_ok(ctx, config);
  if (!valid) return fail(ctx, PCV_ERR_INVALID_ARG, "launch configuration out of range for this context");
  if (ctx->path == PATH_MFMA) TRY(apply_mfma_cfg(ctx, config));
  else if (ctx->path == PATH_VALU_SPLIT) TRY(apply_valu_split_cfg(ctx, config));
  else TRY(apply_waves(ctx, config));
  return PCV_OK;
}

pcv_status pcv_get_launch_config(pcv_ctx ctx, int32_t* config) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (!config) return fail(ctx, PCV_ERR_INVALID_ARG, "null output");
  if (ctx->path == PATH_UNFUSED) return fail(ctx, PCV_ERR_UNSUPPORTED, "the plain fp64 path has no launch shape");
  *config = ctx->path == PATH_MFMA ? MFMA_CFG_SHAPE * ctx->mshape + ctx->n_splits
            : ctx->path == PATH_VALU_SPLIT ? VALU_CFG_WAVES * ctx->W + ctx->n_splits : ctx->W;
  return PCV_OK;
}

// ---- full-data tuning (Section 3.1; workflow Steps 1-2) ----------------------

pcv_status pcv_adapt(pcv_ctx ctx, int64_t n_adapt, double target_accept, double* step_size, double* inv_mass) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  if (n_adapt < 1) return fail(ctx, PCV_ERR_INVALID_ARG, "n_adapt must be >= 1");
  if (!(target_accept > 0.0 && target_accept < 1.0))
    return fail(ctx, PCV_ERR_INVALID_ARG, "target_accept must lie in (0, 1)");
  DevModel& m = ctx->m;
  const int64_t d = m.d, C = m.C;
  // Schedule: initial fast buffer, doubling slow windows (the last stretched
  // to the final buffer), final fast buffer; 75 / 25 / 50, or 15% / rest / 10%
  // of n_adapt when those do not fit.
  int64_t init = 75, term = 50, win = 25;
  if (init + win + term > n_adapt) {
    init = static_cast<int64_t>(0.15 * static_cast<double>(n_adapt));
    term = static_cast<int64_t>(0.1 * static_cast<double>(n_adapt));
    win = n_adapt - init - term;
  }
  std::vector<int64_t> ends;
  if (win > 0) {
    const int64_t last = n_adapt - term;
    for (int64_t start = init, size = win; start < last; size *= 2) {
      int64_t end = start + size;
      if (end + 2 * size > last) end = last;
      ends.push_back(end);
      start = end;
    }
  }
  const int64_t slow_lo = init, slow_hi = ends.empty() ? 0 : ends.back();
  // dual averaging of log eps toward the target acceptance statistic
  const double gamma = 0.05, t0 = 10.0, kappa = 0.75;
  double log_eps = std::log(m.eps), mu = std::log(10.0 * m.eps), hbar = 0.0, log_epsbar = 0.0;
  int64_t mda = 0;
  std::vector<double> alpha(static_cast<size_t>(C)), q(static_cast<size_t>(d * C));
  std::vector<double> mean(static_cast<size_t>(d), 0.0), m2(static_cast<size_t>(d), 0.0), minv(static_cast<size_t>(d));
  int64_t nwin = 0;
  CK(hipMemcpy(minv.data(), m.minv, sizeof(double) * d, hipMemcpyDeviceToHost));
  const bool graphs = ctx->graphs;
  ctx->graphs = false;   // the step size changes every transition: eager launches
  drop_graph(ctx);
  pcv_status st = PCV_OK;
  size_t next_end = 0;
  for (int64_t t = 0; t < n_adapt && st == PCV_OK; ++t) {
    m.eps = std::exp(log_eps);
    st = pcv_step(ctx, 1);
    if (st != PCV_OK) break;
    if (hipMemcpyAsync(alpha.data(), m.acc_stat, sizeof(double) * C, hipMemcpyDeviceToHost, ctx->st) != hipSuccess ||
        hipStreamSynchronize(ctx->st) != hipSuccess) {
      st = fail(ctx, PCV_ERR_DEVICE, "reading the acceptance statistics failed");
      break;
    }
    double a = 0.0;
    for (int64_t c = 0; c < C; ++c) a += alpha[c];
    a /= static_cast<double>(C);
    mda += 1;
    const double w = 1.0 / (static_cast<double>(mda) + t0);
    hbar = (1.0 - w) * hbar + w * (target_accept - a);
    log_eps = mu - std::sqrt(static_cast<double>(mda)) / gamma * hbar;
    const double eta = std::pow(static_cast<double>(mda), -kappa);
    log_epsbar = eta * log_eps + (1.0 - eta) * log_epsbar;
    if (t >= slow_lo && t < slow_hi) {
      // positions of every chain feed a per-coordinate Welford variance
      if (hipMemcpy(q.data(), m.q0, sizeof(double) * d * C, hipMemcpyDeviceToHost) != hipSuccess) {
        st = fail(ctx, PCV_ERR_DEVICE, "reading the positions failed");
        break;
      }
      for (int64_t c = 0; c < C; ++c) {
        nwin += 1;
        for (int64_t j = 0; j < d; ++j) {
          const double x = q[j * C + c];
          const double dx = x - mean[j];
          mean[j] += dx / static_cast<double>(nwin);
          m2[j] += dx * (x - mean[j]);
        }
      }
    }
    if (next_end < ends.size() && t + 1 == ends[next_end]) {
      ++next_end;
      const double nn = static_cast<double>(nwin);
      for (int64_t j = 0; j < d; ++j)
        minv[j] = nn / (nn + 5.0) * (nwin > 1 ? m2[j] / (nn - 1.0) : 0.0) + 1e-3 * 5.0 / (nn + 5.0);
      if (hipMemcpy(const_cast<double*>(m.minv), minv.data(), sizeof(double) * d, hipMemcpyHostToDevice) !=
          hipSuccess) {
        st = fail(ctx, PCV_ERR_DEVICE, "writing the inverse mass failed");
        break;
      }
      std::fill(mean.begin(), mean.end(), 0.0);
      std::fill(m2.begin(), m2.end(), 0.0);
      nwin = 0;
      log_eps = std::log(std::exp(log_eps));     // restart the dual averaging from the current eps
      mu = std::log(10.0 * std::exp(log_eps));
      hbar = 0.0;
      log_epsbar = 0.0;
      mda = 0;
    }
  }
  ctx->graphs = graphs;
  if (st != PCV_OK) return st;
  m.eps = std::exp(log_epsbar);
  drop_graph(ctx);   // a captured transition holds the old step size
  if (step_size) *step_size = m.eps;
  if (inv_mass) std::memcpy(inv_mass, minv.data(), sizeof(double) * d);
  return PCV_OK;
}

pcv_status pcv_init_positions(const double* draws, int64_t n_draws, int64_t d, int64_t C, uint64_t seed,
                              int64_t chain_offset, double* init_pos) {
  if (!draws || !init_pos || n_draws < 1 || d < 1 || C < 1 || chain_offset < 0 ||
      chain_offset + C > 0xFFFFFFFFLL)
    return PCV_ERR_INVALID_ARG;
  const uint32_t k0 = static_cast<uint32_t>(seed & 0xFFFFFFFFu), k1 = static_cast<uint32_t>(seed >> 32);
  for (int64_t c = 0; c < C; ++c) {
    const W4 w = philox4x32_10(W4{static_cast<uint32_t>(chain_offset + c), 0u, TAG_INIT, 0u}, k0, k1);
    const double u = uniform01(w.x, w.y);
    int64_t idx = static_cast<int64_t>(std::floor(u * static_cast<double>(n_draws)));
    if (idx > n_draws - 1) idx = n_draws - 1;
    std::memcpy(init_pos + c * d, draws + idx * d, sizeof(double) * d);
  }
  return PCV_OK;
}

pcv_status pcv_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out) {
  if (n < 0 || (n > 0 && !out)) return PCV_ERR_INVALID_ARG;
  if (n == 0) return PCV_OK;
  uint32_t* d = nullptr;
  if (hipMalloc(&d, sizeof(uint32_t) * 4 * n) != hipSuccess) return PCV_ERR_NOMEM;
  hipError_t e = launch_philox(static_cast<uint32_t>(seed & 0xFFFFFFFFu), static_cast<uint32_t>(seed >> 32), c0, c1,
                               c2, c3, n, d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, d, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? PCV_OK : PCV_ERR_DEVICE;
}

pcv_status pcv_timing_enable(pcv_ctx ctx, int32_t on) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  ctx->timing = on != 0;
  return PCV_OK;
}

pcv_status pcv_timing_read(pcv_ctx ctx, double* ms_sum, int64_t* n_launches, const char** kernel_name,
                           int32_t reset) {
  if (!usable(ctx)) return PCV_ERR_STATE;
  CK(hipStreamSynchronize(ctx->st));
  timing_collect(ctx);
  if (ms_sum) *ms_sum = ctx->ms_acc;
  if (n_launches) *n_launches = ctx->n_launch;
  if (kernel_name)
    *kernel_name = ctx->path == PATH_MFMA && ctx->mshape == MFMA_SHAPE_32X32X16
                       ? "k_mfma32 (bf16 split 32x32x16 MFMA value+gradient)"
                   : ctx->path == PATH_MFMA && ctx->mshape == MFMA_SHAPE_32X32X16_IL
                       ? "k_mfma32 (bf16 split 32x32x16 MFMA value+gradient, free schedule)"
                   : ctx->path == PATH_MFMA && ctx->mshape == MFMA_SHAPE_16X16X32_C16
                       ? "k_mfma (bf16 split 16x16x32 MFMA value+gradient, 16 chains per wave)"
                       : kGradKernelName[ctx->path];
  if (reset) {
    ctx->ms_acc = 0.0;
    ctx->n_launch = 0;
  }
  return PCV_OK;
}

}  // extern "C"
