// Host runtime behind the C ABI of include/pasd.h: validation, device state,
// the iteration driver and checkpoint access.  All numerical work is done by
// the kernels in kernels_*.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "pasd.h"
#include "pasd_internal.hpp"

using namespace pasd;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? PASD_ERR_OOM : PASD_ERR_HIP,             \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

constexpr int kIterChunk = 16;   // iterations enqueued between convergence checks
constexpr int kGraphIters = 16;  // iterations per captured graph

struct Layout {
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t off = total;
    total += (bytes + 255) / 256 * 256;
    return off;
  }
};

int64_t prod_except(const pasd_config* c, int n) {
  int64_t p = 1;
  for (int m = 0; m < c->order; ++m)
    if (m != n) p *= c->dims[m];
  return p;
}

}  // namespace

struct pasd_ctx {
  pasd_config cfg;
  int N = 0;
  int64_t numel = 0;
  int dev = 0;
  hipStream_t stream = nullptr;
  size_t elem = 8;  // bytes per state element
  ModeGeom geom[kMaxN];
  double lam[kMaxN];
  double alpha[kMaxN];
  int mblocks[kMaxN];
  int sblocks[kMaxN];
  void* base = nullptr;
  size_t bytes = 0;
  DevScalars* host_sc = nullptr;  // pinned host mirror
  Problem<float> pf;
  Problem<double> pd;
  Problem<float> vf[kMaxTiles];  // rank-tile views (problems with some R_n > kRT)
  Problem<double> vd[kMaxTiles];
  void* T = nullptr;
  void* scratch_out = nullptr;  // numel elements, for host exports
  // kGraphIters iterations captured once (on cap_stream) and replayed on `stream`
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  bool graph_disabled = false;
  void* dev_prob = nullptr;  // device copy of pd / pf, inside `base`
  // an import changed the iterate: the merged modes' GEMM-M partials are
  // recomputed before the next iteration (see Problem::mmerge)
  bool mrefresh = false;
};

namespace {

int validate_impl(const pasd_config* c) {
  if (!c) return fail(PASD_ERR_INVALID_ARG, "config is NULL");
  if (c->order < 2 || c->order > PASD_MAX_ORDER)
    return fail(PASD_ERR_INVALID_ARG, "order must be in [2, " + std::to_string(PASD_MAX_ORDER) + "]");
  double numel = 1;
  for (int n = 0; n < c->order; ++n) {
    if (c->dims[n] < 1) return fail(PASD_ERR_INVALID_ARG, "dims must be >= 1");
    numel *= (double)c->dims[n];
  }
  if (numel > (double)(1LL << 40)) return fail(PASD_ERR_UNSUPPORTED, "tensor too large");
  for (int n = 0; n < c->order; ++n) {
    const int64_t J = prod_except(c, n);
    const int64_t R = c->ranks[n];
    if (R < 1 || R > c->dims[n] || R > J)
      return fail(PASD_ERR_INVALID_ARG, "rank R_" + std::to_string(n) +
                                            " must satisfy 1 <= R_n <= min(I_n, J_n)");
    if (R > PASD_MAX_RANK)
      return fail(PASD_ERR_UNSUPPORTED, "rank above " + std::to_string(PASD_MAX_RANK));
    if (c->dims[n] > (1 << 30)) return fail(PASD_ERR_UNSUPPORTED, "dimension too large");
    if (c->dims[n] * R > (R <= kRT ? (1 << 20) : 16384))
      return fail(PASD_ERR_UNSUPPORTED, R <= kRT ? "I_n * R_n above 2^20"
                                                 : "I_n * R_n above 16384 (QR workspace)");
    if (!isfinite(c->lambda[n]) || !isfinite(c->alpha[n]))
      return fail(PASD_ERR_INVALID_ARG, "lambda and alpha must be finite");
  }
  if (!(c->mu0 > 0) || !isfinite(c->mu0)) return fail(PASD_ERR_INVALID_ARG, "mu0 must be > 0");
  if (!(c->mu_max >= c->mu0) || !isfinite(c->mu_max))
    return fail(PASD_ERR_INVALID_ARG, "mu_max must be >= mu0");
  if (!(c->rho >= 1.0) || !isfinite(c->rho)) return fail(PASD_ERR_INVALID_ARG, "rho must be >= 1");
  if (!(c->tol >= 0.0) || !isfinite(c->tol)) return fail(PASD_ERR_INVALID_ARG, "tol must be >= 0");
  if (c->max_iter < 1) return fail(PASD_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (c->precision != PASD_FP64 && c->precision != PASD_FP32 && c->precision != PASD_BF16_GEMM)
    return fail(PASD_ERR_INVALID_ARG, "unknown precision");
  if (c->flags & ~(PASD_FLAG_NO_GRAPH | PASD_FLAG_TIEBREAK_KEEP | PASD_FLAG_NO_FLOOR_STOP))
    return fail(PASD_ERR_INVALID_ARG, "unknown flag");
  return PASD_OK;
}

// Buffer plan shared by pasd_footprint and pasd_create.
struct Plan {
  Layout L;
  size_t off_T, off_D, off_sc, off_hist, off_prob, off_views;
  size_t off_Y[kMaxN], off_P[kMaxN], off_U[kMaxN], off_Us[kMaxN], off_Uf[kMaxN], off_UfT[kMaxN],
      off_Mpart[kMaxN], off_M[kMaxN], off_Spart[kMaxN], off_Wf[kMaxN], off_Wev[kMaxN],
      off_Fac[kMaxN];
  ModeGeom geom[kMaxN];
  int mblocks[kMaxN], sblocks[kMaxN];
  int64_t numel;
  // fused pass: vector width of the last mode, 32-bit offsets, blocks, and
  // the modes whose GEMM-M it folds in (merge_plan)
  int vec, idx32, fblocks, mmerge, mfull;
  int64_t mcb;
  size_t off_Mf[kMaxN], off_Mq[kMaxN], off_mcnt[kMaxN];
};

void make_plan(const pasd_config* c, Plan& p, bool own_T = true) {
  const int N = c->order;
  const size_t es = c->precision == PASD_FP64 ? 8 : 4;
  int64_t numel = 1;
  for (int n = 0; n < N; ++n) numel *= c->dims[n];
  p.numel = numel;
  int rmax = 1;
  int64_t span = numel;
  for (int n = 0; n < N; ++n) {
    ModeGeom& g = p.geom[n];
    g.A = 1;
    for (int m = 0; m < n; ++m) g.A *= c->dims[m];
    g.B = 1;
    for (int m = n + 1; m < N; ++m) g.B *= c->dims[m];
    g.I = (int)c->dims[n];
    g.J = g.A * g.B;
    g.R = (int)c->ranks[n];
    g.T = (g.R + kRT - 1) / kRT;
    rmax = std::max(rmax, g.R);
    span = std::max<int64_t>(span, (int64_t)kRT * g.T * g.J);
  }
  const int vw = 16 / (int)es;
  p.vec = (c->dims[N - 1] % vw) == 0 ? vw : 1;
  p.idx32 = span * (int64_t)es < (int64_t(1) << 31) ? 1 : 0;
  merge_plan(c->dims, N, numel, p.vec, rmax, (int)es, p.idx32 != 0, &p.mmerge, &p.mcb, &p.fblocks,
             &p.mfull);
  for (int n = 0; n < N; ++n) {
    // GEMM-M split-K partials, or with mfull the k_msum group sums
    p.mblocks[n] = n < p.mmerge ? 0 : p.mfull ? kMsumGroups : gemm_m_blocks(p.geom[n], N - p.mmerge);
    p.sblocks[n] = gram_blocks(p.geom[n]);
  }
  p.off_T = own_T ? p.L.add(numel * es) : 0;  // T read in place when not owned
  p.off_D = p.L.add(numel * es);
  p.off_sc = p.L.add(sizeof(DevScalars));
  p.off_prob = p.L.add(std::max(sizeof(Problem<float>), sizeof(Problem<double>)));
  p.off_views = p.L.add(kMaxTiles * std::max(sizeof(Problem<float>), sizeof(Problem<double>)));
  p.off_hist = p.L.add(sizeof(double) * (size_t)c->max_iter * N);
  for (int n = 0; n < N; ++n) {
    const ModeGeom& g = p.geom[n];
    const size_t RT = (size_t)g.T * kRT;
    p.off_Y[n] = p.L.add(numel * es);
    p.off_P[n] = p.L.add(RT * g.J * es);  // rows >= R stay zero
    p.off_U[n] = p.L.add((size_t)g.I * g.R * 8);
    p.off_Us[n] = p.L.add((size_t)g.I * RT * es);
    p.off_Uf[n] = p.L.add((size_t)g.I * RT * es);
    p.off_UfT[n] = p.L.add((size_t)g.I * RT * es);
    p.off_Mpart[n] = p.L.add((size_t)p.mblocks[n] * g.I * RT * 8);
    p.off_M[n] = p.L.add((size_t)g.I * RT * 8);
    p.off_Spart[n] = p.L.add((size_t)p.sblocks[n] * RT * RT * 8);
    p.off_Wf[n] = p.L.add(RT * RT * 8);
    p.off_Wev[n] = p.L.add(RT * RT * 8);
    p.off_Fac[n] = p.L.add(RT * 8);
    p.off_Mf[n] = n < p.mmerge ? p.L.add((size_t)p.fblocks * kRT * 8) : 0;
    p.off_Mq[n] = p.mfull && n >= p.mmerge ? p.L.add((size_t)p.fblocks * g.I * g.R * 8) : 0;
    p.off_mcnt[n] = p.mfull && n >= p.mmerge ? p.L.add(((size_t)g.I * g.R + 63) / 64 * 4) : 0;
  }
}

template <typename S>
void fill_problem(pasd_ctx* ctx, const Plan& pl, Problem<S>& p) {
  char* b = static_cast<char*>(ctx->base);
  memset(&p, 0, sizeof(p));
  p.N = ctx->N;
  p.numel = ctx->numel;
  p.T = reinterpret_cast<const S*>(ctx->T);
  p.D = reinterpret_cast<S*>(b + pl.off_D);
  p.sc = reinterpret_cast<DevScalars*>(b + pl.off_sc);
  p.hist = reinterpret_cast<double*>(b + pl.off_hist);
  for (int n = 0; n < ctx->N; ++n) {
    p.g[n] = pl.geom[n];
    ModeBufs<S>& m = p.m[n];
    m.Y = reinterpret_cast<S*>(b + pl.off_Y[n]);
    m.P = reinterpret_cast<S*>(b + pl.off_P[n]);
    m.U = reinterpret_cast<double*>(b + pl.off_U[n]);
    m.Us = reinterpret_cast<S*>(b + pl.off_Us[n]);
    m.Uf = reinterpret_cast<S*>(b + pl.off_Uf[n]);
    m.UfT = reinterpret_cast<S*>(b + pl.off_UfT[n]);
    m.Mpart = reinterpret_cast<double*>(b + pl.off_Mpart[n]);
    m.M = reinterpret_cast<double*>(b + pl.off_M[n]);
    m.Spart = reinterpret_cast<double*>(b + pl.off_Spart[n]);
    m.Wf = reinterpret_cast<double*>(b + pl.off_Wf[n]);
    m.Wev = reinterpret_cast<double*>(b + pl.off_Wev[n]);
    m.Fac = reinterpret_cast<double*>(b + pl.off_Fac[n]);
    m.Mf = n < pl.mmerge ? reinterpret_cast<double*>(b + pl.off_Mf[n]) : nullptr;
    m.Mq = pl.mfull && n >= pl.mmerge ? reinterpret_cast<double*>(b + pl.off_Mq[n]) : nullptr;
    m.mcnt = pl.mfull && n >= pl.mmerge ? reinterpret_cast<unsigned int*>(b + pl.off_mcnt[n]) : nullptr;
    m.mblocks = pl.mblocks[n];
    m.sblocks = pl.sblocks[n];
    p.lam[n] = ctx->lam[n];
    p.alpha[n] = ctx->alpha[n];
  }
  p.mu_max = ctx->cfg.mu_max;
  p.rho = ctx->cfg.rho;
  p.tol = ctx->cfg.tol;
  p.max_iter = ctx->cfg.max_iter;
  p.precision = ctx->cfg.precision;
  p.tiebreak_keep = (ctx->cfg.flags & PASD_FLAG_TIEBREAK_KEEP) != 0 ? 1 : 0;
  p.floor_stop = (ctx->cfg.flags & PASD_FLAG_NO_FLOOR_STOP) != 0 ? 0 : 1;
  // per-mode block offsets of the mode-grouped kernels, and the fused-pass share
  for (int n = 0; n <= ctx->N; ++n)
    for (int k = 0; k < KB_COUNT; ++k) p.kb[k][n] = 0;
  {
    // GEMM-P of the last two modes as one pass over their 64 x 64 slabs
    const int N = ctx->N;
    bool narrow = true;
    for (int n = 0; n < N; ++n) narrow = narrow && p.g[n].R <= kRT;
    // (not with split-BF16 operands: the splitting doubles the pass's
    // registers, and there it was measured slower, 135 -> 142 us at 64^4)
    p.gp2 = (N >= 3 && narrow && p.g[N - 1].I == 64 && p.g[N - 2].I == 64 &&
             p.precision != PASD_BF16_GEMM)
                ? (int)p.g[N - 2].A
                : 0;
  }
  for (int n = 0; n < ctx->N; ++n) {
    const ModeGeom& g = p.g[n];
    p.kb[KB_GEMM_M][n + 1] = p.kb[KB_GEMM_M][n] + (pl.mfull ? 0 : p.m[n].mblocks);
    p.kb[KB_MSUM][n + 1] = p.kb[KB_MSUM][n] +
                           (!pl.mfull ? 0 : n >= pl.mmerge ? msum_blocks(g) : reduce_m_blocks(g));
    p.kb[KB_REDUCE_M][n + 1] = p.kb[KB_REDUCE_M][n] + reduce_m_blocks(g);
    p.kb[KB_GEMM_P][n + 1] = p.kb[KB_GEMM_P][n] + (p.gp2 && n >= ctx->N - 2 ? 0 : gemm_p_blocks(g));
    p.kb[KB_GRAM][n + 1] = p.kb[KB_GRAM][n] + p.m[n].sblocks;
  }
  const int vw = 16 / (int)sizeof(S);
  p.vecw = pl.vec == vw ? 1 : 0;
  p.fused_blocks = pl.fblocks;
  // 32-bit offsets in the fused pass when every element offset, and every
  // index divided there, stays below 2^31 bytes
  p.idx32 = pl.idx32;
  p.mmerge = pl.mmerge;
  p.mfull = pl.mfull;
  p.ntstore = (int64_t)(ctx->N + 1) * ctx->numel * (int64_t)sizeof(S) > (int64_t(256) << 20) ? 1 : 0;
  p.mcb = (uint32_t)pl.mcb;
  for (int n = 0; n < kMaxN; ++n)
    p.mslab[n] = n < pl.mmerge ? (int)(p.g[n].B / pl.vec / pl.mcb) : 0;
  const int64_t IN = p.g[ctx->N - 1].I;
  p.fd_q = make_fastdiv((uint32_t)(p.idx32 ? IN / (p.vecw ? vw : 1) : 1));
  // Mode-1 order of the fused pass when P_0 would not stay in one XCD's L2
  // (4 MB, shared with the streamed tensors): more than 2 MiB of P_0.
  const int64_t vec = p.vecw ? vw : 1;
  const int64_t p0_bytes = (int64_t)p.g[0].R * p.g[0].J * (int64_t)sizeof(S);
  p.fsplit1 = (p.mmerge == 0 && ctx->N >= 3 && p.idx32 && p.g[1].I % kXcds == 0 &&
               p0_bytes > (int64_t(2) << 20)) ? 1 : 0;
  p.f_cp1 = p.fsplit1 ? (uint32_t)(p.g[1].B / vec) : 1;
  p.f_cp0 = p.fsplit1 ? (uint32_t)(p.g[0].B / vec) : 1;
  p.f_seg = p.fsplit1 ? p.f_cp1 * (uint32_t)(p.g[1].I / kXcds) : 1;
  p.fd_seg = make_fastdiv(p.f_seg);
  for (int n = 0; n < kMaxN; ++n) {
    const bool inner = n < ctx->N - 1 && p.idx32;
    p.fd_rb[n] = make_fastdiv((uint32_t)(inner ? p.g[n].B / IN : 1));
    p.fd_i[n] = make_fastdiv((uint32_t)(inner ? p.g[n].I : 1));
    p.fd_b[n] = make_fastdiv((uint32_t)(n < ctx->N && p.g[n].B < (int64_t(1) << 31) ? p.g[n].B : 1));
  }
}

// Rank-tile views of a problem with some R_n > kRT (see Problem::wide): view t
// keeps, for every mode with R_n > kRT t, tile t of the rank-indexed buffers
// the unfolding GEMMs and the GEMM-M reduction touch, with R_n replaced by the
// tile's R_t <= kRT; the other modes get no blocks.  Device copies follow the
// problem's own in the allocation.
template <typename S>
void fill_views(pasd_ctx* ctx, const Plan& pl, Problem<S>& p, Problem<S>* views) {
  int T = 1;
  for (int n = 0; n < p.N; ++n) T = std::max(T, p.g[n].T);
  p.wide = T > 1 ? 1 : 0;
  p.ntiles = T;
  for (int t = 0; t < kMaxTiles; ++t) {
    p.view_host[t] = nullptr;
    p.view_dev[t] = nullptr;
  }
  if (!p.wide) return;
  char* dv = static_cast<char*>(ctx->base) + pl.off_views;
  for (int t = 0; t < T; ++t) {
    Problem<S>& v = views[t];
    v = p;
    v.wide = 0;
    v.ntiles = 1;
    v.gp2 = 0;
    for (int u = 0; u < kMaxTiles; ++u) {
      v.view_host[u] = nullptr;
      v.view_dev[u] = nullptr;
    }
    for (int k = 0; k < KB_COUNT; ++k) v.kb[k][0] = 0;
    for (int n = 0; n < p.N; ++n) {
      ModeGeom& g = v.g[n];
      ModeBufs<S>& m = v.m[n];
      const int Rt = std::min(kRT, p.g[n].R - kRT * t);
      const bool has = Rt > 0;
      if (has) {
        g.R = Rt;
        g.T = 1;
        m.P += (int64_t)kRT * t * g.J;
        m.Us += (int64_t)t * g.I * kRT;
        m.Mpart += (int64_t)t * m.mblocks * g.I * kRT;
        m.M += (int64_t)t * g.I * kRT;
      }
      v.kb[KB_GEMM_M][n + 1] = v.kb[KB_GEMM_M][n] + (has ? m.mblocks : 0);
      v.kb[KB_REDUCE_M][n + 1] = v.kb[KB_REDUCE_M][n] + (has ? reduce_m_blocks(g) : 0);
      v.kb[KB_GEMM_P][n + 1] = v.kb[KB_GEMM_P][n] + (has ? gemm_p_blocks(g) : 0);
      v.kb[KB_GRAM][n + 1] = v.kb[KB_GRAM][n];
      v.kb[KB_MSUM][n + 1] = v.kb[KB_MSUM][n];
    }
    p.view_host[t] = &v;
    p.view_dev[t] = reinterpret_cast<const Problem<S>*>(dv + (size_t)t * sizeof(Problem<S>));
  }
}

template <typename S>
hipError_t upload_problem(pasd_ctx* ctx, const Problem<S>& p) {
  hipError_t e = hipMemcpyAsync(ctx->dev_prob, &p, sizeof(p), hipMemcpyHostToDevice, ctx->stream);
  for (int t = 0; e == hipSuccess && p.wide && t < p.ntiles; ++t)
    e = hipMemcpyAsync(const_cast<Problem<S>*>(p.view_dev[t]), p.view_host[t], sizeof(p),
                       hipMemcpyHostToDevice, ctx->stream);
  return e;
}

// Enqueue `count` iterations; with `ev` non-null an event is recorded before
// the first launch and after every launch (ev[it * PASD_NUM_KERNELS + k + 1]).
template <typename S>
void enqueue_iterations(const LaunchSet<S>& p, int count, hipStream_t s, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], s);
  for (int it = 0; it < count; ++it) {
    hipEvent_t* e = ev ? ev + (size_t)it * PASD_NUM_KERNELS + 1 : nullptr;
    launch_gemm_m<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_GEMM_M], s);
    launch_reduce_m<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_REDUCE_M], s);
    launch_qr<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_QR], s);
    launch_gemm_p<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_GEMM_P], s);
    launch_gram<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_GRAM], s);
    launch_eig<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_EIG], s);
    launch_fused<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_FUSED], s);
    launch_control<S>(p, s);
    if (e) (void)hipEventRecord(e[PASD_K_CONTROL], s);
  }
}

void enqueue_direct(pasd_ctx* ctx, int count, hipStream_t s, hipEvent_t* ev) {
  if (ctx->cfg.precision == PASD_FP64) {
    LaunchSet<double> ls;
    ls.count = 1;
    ls.host[0] = &ctx->pd;
    ls.dev[0] = static_cast<const Problem<double>*>(ctx->dev_prob);
    enqueue_iterations<double>(ls, count, s, ev);
  } else {
    LaunchSet<float> ls;
    ls.count = 1;
    ls.host[0] = &ctx->pf;
    ls.dev[0] = static_cast<const Problem<float>*>(ctx->dev_prob);
    enqueue_iterations<float>(ls, count, s, ev);
  }
}

// Capture kGraphIters iterations into a graph once.  Capture needs a stream
// other than the legacy null stream, so it runs on a private non-blocking
// stream; the graph is then launched on the context's stream.  Any failure
// leaves the context on direct launches.
void ensure_graph(pasd_ctx* ctx) {
  if (ctx->graph || ctx->graph_disabled) return;
  ctx->graph_disabled = true;
  if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    ctx->cap_stream = nullptr;
    return;
  }
  if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return;
  enqueue_direct(ctx, kGraphIters, ctx->cap_stream, nullptr);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(ctx->cap_stream, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess || !ex) {
    (void)hipGetLastError();
    return;
  }
  ctx->graph = ex;
  ctx->graph_disabled = false;
}

// After an import, the merged modes' GEMM-M partials of the restored iterate
// (launched directly, never captured).
void refresh_merged(pasd_ctx* ctx, hipStream_t s) {
  if (!ctx->mrefresh) return;
  ctx->mrefresh = false;
  if (ctx->cfg.precision == PASD_FP64) {
    if (!ctx->pd.mmerge) return;
    LaunchSet<double> ls;
    ls.count = 1;
    ls.host[0] = &ctx->pd;
    ls.dev[0] = static_cast<const Problem<double>*>(ctx->dev_prob);
    launch_mrefresh<double>(ls, s);
  } else {
    if (!ctx->pf.mmerge) return;
    LaunchSet<float> ls;
    ls.count = 1;
    ls.host[0] = &ctx->pf;
    ls.dev[0] = static_cast<const Problem<float>*>(ctx->dev_prob);
    launch_mrefresh<float>(ls, s);
  }
}

int enqueue(pasd_ctx* ctx, int count, hipEvent_t* ev = nullptr) {
  if (count > 0) refresh_merged(ctx, ctx->stream);
  // The graph is captured and instantiated on the first enqueue of any
  // length, so that a caller's warm-up (even one iteration) absorbs that cost
  // and later calls replay it.
  if (!ev && count > 0 && !ctx->graph_disabled) {
    ensure_graph(ctx);
    if (ctx->graph) {
      for (; count >= kGraphIters; count -= kGraphIters)
        HIP_TRY(hipGraphLaunch(ctx->graph, ctx->stream));
    }
  }
  if (count > 0) enqueue_direct(ctx, count, ctx->stream, ev);
  HIP_TRY(hipGetLastError());
  return PASD_OK;
}

int read_scalars(pasd_ctx* ctx) {
  DevScalars* dsc = ctx->cfg.precision == PASD_FP64 ? ctx->pd.sc : ctx->pf.sc;
  HIP_TRY(hipMemcpyAsync(ctx->host_sc, dsc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PASD_OK;
}

void fill_info(pasd_ctx* ctx, pasd_info* info) {
  memset(info, 0, sizeof(*info));
  const DevScalars* s = ctx->host_sc;
  info->iterations = s->k;
  info->converged = s->converged;
  info->done = s->done;
  info->mu = s->mu;
  for (int n = 0; n < ctx->N; ++n) {
    info->residual[n] = s->residual[n];
    info->rank[n] = s->rank[n];
    info->eig_sweeps[n] = s->eig_sweeps[n];
    info->tol_effective = s->tol_eff;
  }
  info->bytes_resident = ctx->bytes;
  // modes whose GEMM-M the fused pass accumulates: 0 .. mmerge-1, and with
  // mfull every mode
  if (ctx->cfg.precision == PASD_FP64) {
    info->merged_modes = ctx->pd.mfull ? ctx->N : ctx->pd.mmerge;
    info->fused_blocks = ctx->pd.fused_blocks;
    info->gemm_p_pair = ctx->pd.gp2 ? 1 : 0;
  } else {
    info->merged_modes = ctx->pf.mfull ? ctx->N : ctx->pf.mmerge;
    info->fused_blocks = ctx->pf.fused_blocks;
    info->gemm_p_pair = ctx->pf.gp2 ? 1 : 0;
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int copy_kind(int on_device) { return on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }

}  // namespace

namespace {

// Host part of a context: configuration, geometry, weights, device and
// stream; touches no device.
int ctx_init_host(pasd_ctx* ctx, const pasd_config* cfg, const Plan& pl) {
  ctx->cfg = *cfg;
  ctx->N = cfg->order;
  int dev = cfg->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(PASD_ERR_HIP, "hipGetDevice failed (no GPU?)");
  ctx->dev = dev;
  ctx->stream = static_cast<hipStream_t>(cfg->stream);
  ctx->graph_disabled = (cfg->flags & PASD_FLAG_NO_GRAPH) != 0;
  ctx->elem = cfg->precision == PASD_FP64 ? 8 : 4;
  ctx->numel = pl.numel;
  for (int n = 0; n < ctx->N; ++n) {
    const double J = (double)prod_except(cfg, n);
    ctx->geom[n] = pl.geom[n];
    ctx->lam[n] = cfg->lambda[n] > 0 ? cfg->lambda[n]
                                     : sqrt(std::max((double)cfg->dims[n], J)) / ctx->N;
    ctx->mblocks[n] = pl.mblocks[n];
    ctx->sblocks[n] = pl.sblocks[n];
  }
  for (int n = 0; n < ctx->N; ++n) ctx->alpha[n] = cfg->alpha[n] > 0 ? cfg->alpha[n] : ctx->lam[n];
  return PASD_OK;
}

// Zero `bytes` (a multiple of 16, 16-byte aligned) with a plain kernel rather
// than a memset node, so that the clearing is an ordinary launch wherever the
// caller's stream is.
__global__ void __launch_bounds__(256) k_zero(uint4* p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = uint4{0u, 0u, 0u, 0u};
}

hipError_t zero_async(void* p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  const size_t blocks = std::min<size_t>(std::max<size_t>(1, (n16 + 255) / 256), 4096);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint4*>(p), n16);
  return hipGetLastError();
}

// Device part: lay the solver state out in `base` (pl.L.total bytes of device
// memory of ctx->dev), clear it, upload the descriptors, bring T in (copied
// into the plan's T slot, or read in place from the caller's device buffer
// when T_in_place) and run the initialisation of Algorithm 1.  Asynchronous
// on ctx->stream.
int ctx_init_device(pasd_ctx* ctx, const Plan& pl, void* base, const void* T, int T_on_device,
                    bool T_in_place) {
  ctx->base = base;
  ctx->T = T_in_place ? const_cast<void*>(T) : static_cast<char*>(base) + pl.off_T;
  // zero the whole state once: the padding rows of P_n and columns of the
  // factors are read by the unrolled kernels and must stay zero
  hipError_t e = zero_async(base, pl.L.total, ctx->stream);
  if (e != hipSuccess) return fail(PASD_ERR_HIP, std::string("clearing state: ") + hipGetErrorString(e));
  ctx->dev_prob = static_cast<char*>(base) + pl.off_prob;
  if (ctx->cfg.precision == PASD_FP64) {
    fill_problem<double>(ctx, pl, ctx->pd);
    fill_views<double>(ctx, pl, ctx->pd, ctx->vd);
    e = upload_problem<double>(ctx, ctx->pd);
  } else {
    fill_problem<float>(ctx, pl, ctx->pf);
    fill_views<float>(ctx, pl, ctx->pf, ctx->vf);
    e = upload_problem<float>(ctx, ctx->pf);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(PASD_ERR_HIP, std::string("problem upload: ") + hipGetErrorString(e));
  if (!T_in_place) {
    e = hipMemcpyAsync(ctx->T, T, (size_t)ctx->numel * ctx->elem,
                       (hipMemcpyKind)copy_kind(T_on_device), ctx->stream);
    if (e != hipSuccess) return fail(PASD_ERR_HIP, std::string("copy of T: ") + hipGetErrorString(e));
  }
  if (ctx->cfg.precision == PASD_FP64)
    launch_init<double>(ctx->pd, ctx->cfg.mu0, ctx->stream);
  else
    launch_init<float>(ctx->pf, ctx->cfg.mu0, ctx->stream);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(PASD_ERR_HIP, std::string("initialisation: ") + hipGetErrorString(e));
  return PASD_OK;
}

}  // namespace

extern "C" {

int pasd_config_init(pasd_config* cfg) {
  if (!cfg) return fail(PASD_ERR_INVALID_ARG, "config is NULL");
  memset(cfg, 0, sizeof(*cfg));
  cfg->mu0 = 1e-4;
  cfg->mu_max = 1e10;
  cfg->rho = 1.1;
  cfg->tol = 1e-5;
  cfg->max_iter = 1000;
  cfg->precision = PASD_FP64;
  cfg->device = -1;
  cfg->stream = nullptr;
  return PASD_OK;
}

int pasd_validate(const pasd_config* cfg) {
  g_last_error.clear();
  return validate_impl(cfg);
}

int pasd_footprint(const pasd_config* cfg, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(PASD_ERR_INVALID_ARG, "bytes is NULL");
  const int rc = validate_impl(cfg);
  if (rc != PASD_OK) return rc;
  Plan pl;
  make_plan(cfg, pl);
  *bytes = pl.L.total + (size_t)pl.numel * (cfg->precision == PASD_FP64 ? 8 : 4);
  return PASD_OK;
}

int pasd_create(const pasd_config* cfg, const void* T, int T_on_device, pasd_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(PASD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate_impl(cfg);
  if (rc != PASD_OK) return rc;
  if (!T) return fail(PASD_ERR_INVALID_ARG, "T is NULL");
  pasd_ctx* ctx = new pasd_ctx();
  Plan pl;
  make_plan(cfg, pl);
  rc = ctx_init_host(ctx, cfg, pl);
  if (rc != PASD_OK) {
    delete ctx;
    return rc;
  }
  DeviceGuard guard(ctx->dev);
  hipError_t e = hipMalloc(&ctx->base, pl.L.total);
  if (e != hipSuccess) {
    delete ctx;
    return fail(e == hipErrorOutOfMemory ? PASD_ERR_OOM : PASD_ERR_HIP,
                std::string("hipMalloc of solver state: ") + hipGetErrorString(e));
  }
  e = hipMalloc(&ctx->scratch_out, (size_t)ctx->numel * ctx->elem);
  if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->host_sc, sizeof(DevScalars), hipHostMallocDefault);
  if (e != hipSuccess) {
    pasd_destroy(ctx);
    return fail(e == hipErrorOutOfMemory ? PASD_ERR_OOM : PASD_ERR_HIP,
                std::string("allocation: ") + hipGetErrorString(e));
  }
  ctx->bytes = pl.L.total + (size_t)ctx->numel * ctx->elem;
  rc = ctx_init_device(ctx, pl, ctx->base, T, T_on_device, false);
  if (rc == PASD_OK) {
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = fail(PASD_ERR_HIP, std::string("create: ") + hipGetErrorString(e));
  }
  if (rc != PASD_OK) {
    pasd_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return PASD_OK;
}

int pasd_reset(pasd_ctx* ctx) {
  if (!ctx) return fail(PASD_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard guard(ctx->dev);
  if (ctx->cfg.precision == PASD_FP64)
    launch_init<double>(ctx->pd, ctx->cfg.mu0, ctx->stream);
  else
    launch_init<float>(ctx->pf, ctx->cfg.mu0, ctx->stream);
  HIP_TRY(hipGetLastError());
  return PASD_OK;
}

int pasd_step(pasd_ctx* ctx, int n_iters) {
  g_last_error.clear();
  if (!ctx) return fail(PASD_ERR_INVALID_ARG, "ctx is NULL");
  if (n_iters < 0) return fail(PASD_ERR_INVALID_ARG, "n_iters must be >= 0");
  DeviceGuard guard(ctx->dev);
  return enqueue(ctx, n_iters);
}

int pasd_query(pasd_ctx* ctx, pasd_info* info) {
  g_last_error.clear();
  if (!ctx || !info) return fail(PASD_ERR_INVALID_ARG, "ctx or info is NULL");
  DeviceGuard guard(ctx->dev);
  int rc = read_scalars(ctx);
  if (rc != PASD_OK) return rc;
  fill_info(ctx, info);
  return PASD_OK;
}

int pasd_solve(pasd_ctx* ctx, pasd_info* info) {
  g_last_error.clear();
  if (!ctx) return fail(PASD_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard guard(ctx->dev);
  for (;;) {
    int rc = read_scalars(ctx);
    if (rc != PASD_OK) return rc;
    if (ctx->host_sc->done) break;
    const int left = ctx->cfg.max_iter - ctx->host_sc->k;
    rc = enqueue(ctx, std::max(1, std::min(kIterChunk, left)));
    if (rc != PASD_OK) return rc;
  }
  if (info) fill_info(ctx, info);
  switch (ctx->host_sc->done) {
    case 1: return PASD_OK;
    case 2: return PASD_NOT_CONVERGED;
    case 4: return PASD_PRECISION_FLOOR;
    default: return fail(PASD_ERR_NUMERIC, "NaN or infinity in the iteration");
  }
}

int pasd_get_result(pasd_ctx* ctx, void* X, void* E, int on_device) {
  g_last_error.clear();
  if (!ctx) return fail(PASD_ERR_INVALID_ARG, "ctx is NULL");
  DeviceGuard guard(ctx->dev);
  const size_t bytes = (size_t)ctx->numel * ctx->elem;
  for (int which = 0; which < 2; ++which) {
    void* dst = which == 0 ? X : E;
    if (!dst) continue;
    void* tgt = on_device ? dst : ctx->scratch_out;
    if (ctx->cfg.precision == PASD_FP64)
      launch_output<double>(ctx->pd, which == 0 ? (double*)tgt : nullptr,
                            which == 1 ? (double*)tgt : nullptr, ctx->stream);
    else
      launch_output<float>(ctx->pf, which == 0 ? (float*)tgt : nullptr,
                           which == 1 ? (float*)tgt : nullptr, ctx->stream);
    HIP_TRY(hipGetLastError());
    if (!on_device)
      HIP_TRY(hipMemcpyAsync(dst, ctx->scratch_out, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  return PASD_OK;
}

int pasd_export(pasd_ctx* ctx, int q, int index, void* dst, int on_device) {
  g_last_error.clear();
  if (!ctx || !dst) return fail(PASD_ERR_INVALID_ARG, "ctx or dst is NULL");
  const bool per_mode = q == PASD_Q_Y || q == PASD_Q_Z || q == PASD_Q_U || q == PASD_Q_P ||
                        q == PASD_Q_UF || q == PASD_Q_WEV || q == PASD_Q_FAC;
  if (per_mode && (index < 0 || index >= ctx->N)) return fail(PASD_ERR_INVALID_ARG, "mode index out of range");
  DeviceGuard guard(ctx->dev);
  const bool f64 = ctx->cfg.precision == PASD_FP64;
  const size_t es = ctx->elem;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const void* src = nullptr;
  size_t bytes = 0;
  switch (q) {
    case PASD_Q_E:
    case PASD_Q_X:
      HIP_TRY(hipStreamSynchronize(ctx->stream));
      return q == PASD_Q_E ? pasd_get_result(ctx, nullptr, dst, on_device)
                           : pasd_get_result(ctx, dst, nullptr, on_device);
    case PASD_Q_Y:
      src = f64 ? (const void*)ctx->pd.m[index].Y : (const void*)ctx->pf.m[index].Y;
      bytes = (size_t)ctx->numel * es;
      break;
    case PASD_Q_D:
      src = f64 ? (const void*)ctx->pd.D : (const void*)ctx->pf.D;
      bytes = (size_t)ctx->numel * es;
      break;
    case PASD_Q_Z: {
      void* tgt = on_device ? dst : ctx->scratch_out;
      if (f64)
        launch_component<double>(ctx->pd, index, (double*)tgt, ctx->stream);
      else
        launch_component<float>(ctx->pf, index, (float*)tgt, ctx->stream);
      HIP_TRY(hipGetLastError());
      if (on_device) {
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return PASD_OK;
      }
      src = ctx->scratch_out;
      bytes = (size_t)ctx->numel * es;
      break;
    }
    case PASD_Q_U:
      src = f64 ? (const void*)ctx->pd.m[index].U : (const void*)ctx->pf.m[index].U;
      bytes = (size_t)ctx->geom[index].I * ctx->geom[index].R * 8;
      break;
    case PASD_Q_P:
      src = f64 ? (const void*)ctx->pd.m[index].P : (const void*)ctx->pf.m[index].P;
      bytes = (size_t)ctx->geom[index].R * ctx->geom[index].J * es;
      break;
    case PASD_Q_UF: {
      // [T][I][kRT] padded state-type copy -> I x R double
      const ModeGeom& g = ctx->geom[index];
      std::vector<char> tmp((size_t)g.I * kRT * g.T * es);
      const void* s = f64 ? (const void*)ctx->pd.m[index].Uf : (const void*)ctx->pf.m[index].Uf;
      HIP_TRY(hipMemcpyAsync(tmp.data(), s, tmp.size(), hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(hipStreamSynchronize(ctx->stream));
      std::vector<double> outv((size_t)g.I * g.R);
      for (int i = 0; i < g.I; ++i)
        for (int r = 0; r < g.R; ++r) {
          const size_t at = ((size_t)(r / kRT) * g.I + i) * kRT + r % kRT;
          outv[(size_t)i * g.R + r] = f64 ? ((const double*)tmp.data())[at]
                                          : (double)((const float*)tmp.data())[at];
        }
      HIP_TRY(hipMemcpy(dst, outv.data(), outv.size() * 8,
                        on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
      return PASD_OK;
    }
    case PASD_Q_WEV: {
      const int R = ctx->geom[index].R, RT = ctx->geom[index].T * kRT;
      std::vector<double> w((size_t)RT * RT), out((size_t)R * R);
      const double* s = f64 ? ctx->pd.m[index].Wev : ctx->pf.m[index].Wev;
      HIP_TRY(hipMemcpyAsync(w.data(), s, w.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(hipStreamSynchronize(ctx->stream));
      for (int r = 0; r < R; ++r)
        for (int c = 0; c < R; ++c) out[(size_t)r * R + c] = w[(size_t)r * RT + c];
      HIP_TRY(hipMemcpy(dst, out.data(), out.size() * 8,
                        on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
      return PASD_OK;
    }
    case PASD_Q_FAC: {
      const int R = ctx->geom[index].R;
      std::vector<double> f(R);
      const double* s = f64 ? ctx->pd.m[index].Fac : ctx->pf.m[index].Fac;
      HIP_TRY(hipMemcpyAsync(f.data(), s, f.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(hipStreamSynchronize(ctx->stream));
      HIP_TRY(hipMemcpy(dst, f.data(), f.size() * 8,
                        on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
      return PASD_OK;
    }
    case PASD_Q_SCALARS: {
      int rc = read_scalars(ctx);
      if (rc != PASD_OK) return rc;
      double v[2] = {(double)ctx->host_sc->k, ctx->host_sc->mu};
      HIP_TRY(hipMemcpy(dst, v, sizeof(v), on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
      return PASD_OK;
    }
    default:
      return fail(PASD_ERR_INVALID_ARG, "unknown quantity");
  }
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, kind, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PASD_OK;
}

int pasd_import(pasd_ctx* ctx, int q, int index, const void* src, int on_device) {
  g_last_error.clear();
  if (!ctx || !src) return fail(PASD_ERR_INVALID_ARG, "ctx or src is NULL");
  const bool per_mode = q == PASD_Q_Y || q == PASD_Q_U || q == PASD_Q_P || q == PASD_Q_WEV ||
                        q == PASD_Q_FAC;
  if (per_mode && (index < 0 || index >= ctx->N)) return fail(PASD_ERR_INVALID_ARG, "mode index out of range");
  DeviceGuard guard(ctx->dev);
  const bool f64 = ctx->cfg.precision == PASD_FP64;
  const size_t es = ctx->elem;
  const hipMemcpyKind kind = (hipMemcpyKind)copy_kind(on_device);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->mrefresh = true;
  switch (q) {
    case PASD_Q_E: {
      // D = T - E, computed on the host side of the copy to keep one code path
      const size_t bytes = (size_t)ctx->numel * es;
      std::vector<char> e(bytes), t(bytes);
      HIP_TRY(hipMemcpy(e.data(), src, bytes, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
      HIP_TRY(hipMemcpy(t.data(), ctx->T, bytes, hipMemcpyDeviceToHost));
      for (int64_t x = 0; x < ctx->numel; ++x) {
        if (f64)
          ((double*)e.data())[x] = ((double*)t.data())[x] - ((double*)e.data())[x];
        else
          ((float*)e.data())[x] = ((float*)t.data())[x] - ((float*)e.data())[x];
      }
      void* D = f64 ? (void*)ctx->pd.D : (void*)ctx->pf.D;
      HIP_TRY(hipMemcpy(D, e.data(), bytes, hipMemcpyHostToDevice));
      return PASD_OK;
    }
    case PASD_Q_Y: {
      void* d = f64 ? (void*)ctx->pd.m[index].Y : (void*)ctx->pf.m[index].Y;
      HIP_TRY(hipMemcpy(d, src, (size_t)ctx->numel * es, kind));
      return PASD_OK;
    }
    case PASD_Q_D: {
      void* d = f64 ? (void*)ctx->pd.D : (void*)ctx->pf.D;
      HIP_TRY(hipMemcpy(d, src, (size_t)ctx->numel * es, kind));
      return PASD_OK;
    }
    case PASD_Q_U: {
      const ModeGeom& g = ctx->geom[index];
      std::vector<double> u((size_t)g.I * g.R);
      HIP_TRY(hipMemcpy(u.data(), src, u.size() * 8, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
      void* d = f64 ? (void*)ctx->pd.m[index].U : (void*)ctx->pf.m[index].U;
      HIP_TRY(hipMemcpy(d, u.data(), u.size() * 8, hipMemcpyHostToDevice));
      std::vector<char> us((size_t)g.I * kRT * g.T * es, 0);
      for (int i = 0; i < g.I; ++i)
        for (int r = 0; r < g.R; ++r) {
          const size_t at = ((size_t)(r / kRT) * g.I + i) * kRT + r % kRT;
          if (f64)
            ((double*)us.data())[at] = u[(size_t)i * g.R + r];
          else
            ((float*)us.data())[at] = (float)u[(size_t)i * g.R + r];
        }
      void* ds = f64 ? (void*)ctx->pd.m[index].Us : (void*)ctx->pf.m[index].Us;
      HIP_TRY(hipMemcpy(ds, us.data(), us.size(), hipMemcpyHostToDevice));
      return PASD_OK;
    }
    case PASD_Q_P: {
      void* d = f64 ? (void*)ctx->pd.m[index].P : (void*)ctx->pf.m[index].P;
      HIP_TRY(hipMemcpy(d, src, (size_t)ctx->geom[index].R * ctx->geom[index].J * es, kind));
      return PASD_OK;
    }
    case PASD_Q_WEV: {
      const int R = ctx->geom[index].R, RT = ctx->geom[index].T * kRT;
      std::vector<double> in((size_t)R * R), w((size_t)RT * RT);
      HIP_TRY(hipMemcpy(in.data(), src, in.size() * 8,
                        on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
      for (int r = 0; r < RT; ++r)
        for (int c = 0; c < RT; ++c)
          w[(size_t)r * RT + c] = (r < R && c < R) ? in[(size_t)r * R + c] : (r == c ? 1.0 : 0.0);
      double* d = f64 ? ctx->pd.m[index].Wev : ctx->pf.m[index].Wev;
      HIP_TRY(hipMemcpy(d, w.data(), w.size() * 8, hipMemcpyHostToDevice));
      return PASD_OK;
    }
    case PASD_Q_FAC: {
      const int R = ctx->geom[index].R;
      std::vector<double> f((size_t)ctx->geom[index].T * kRT, 0.0);
      HIP_TRY(hipMemcpy(f.data(), src, sizeof(double) * R,
                        on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
      double* d = f64 ? ctx->pd.m[index].Fac : ctx->pf.m[index].Fac;
      HIP_TRY(hipMemcpy(d, f.data(), f.size() * 8, hipMemcpyHostToDevice));
      return PASD_OK;
    }
    case PASD_Q_SCALARS: {
      double v[2];
      HIP_TRY(hipMemcpy(v, src, sizeof(v), on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
      if (!(v[1] > 0) || v[0] < 0 || v[0] > ctx->cfg.max_iter)
        return fail(PASD_ERR_INVALID_ARG, "scalars must hold 0 <= k <= max_iter and mu > 0");
      int rc = read_scalars(ctx);
      if (rc != PASD_OK) return rc;
      DevScalars s = *ctx->host_sc;
      s.k = (int)v[0];
      s.mu = v[1];
      s.done = s.k >= ctx->cfg.max_iter ? 2 : 0;
      s.converged = 0;
      for (int n = 0; n <= kMaxN; ++n)
        for (int b = 0; b < kResSlots; ++b) s.res_slots[n][b] = 0;
      DevScalars* dsc = f64 ? ctx->pd.sc : ctx->pf.sc;
      HIP_TRY(hipMemcpy(dsc, &s, sizeof(s), hipMemcpyHostToDevice));
      return PASD_OK;
    }
    default:
      return fail(PASD_ERR_INVALID_ARG, "quantity cannot be imported");
  }
}

}  // extern "C"

namespace {

int check_batch(pasd_ctx* const* ctxs, int count, int n_iters) {
  if (count < 0 || (count > 0 && !ctxs)) return fail(PASD_ERR_INVALID_ARG, "bad context list");
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return fail(PASD_ERR_INVALID_ARG, "NULL context in batch");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(PASD_ERR_INVALID_ARG, "context repeated in batch");
    if (ctxs[i]->dev != ctxs[0]->dev) return fail(PASD_ERR_INVALID_ARG, "contexts on different devices");
    if (ctxs[i]->stream != ctxs[0]->stream)
      return fail(PASD_ERR_INVALID_ARG, "contexts of a batch must share one stream");
  }
  if (n_iters < 0) return fail(PASD_ERR_INVALID_ARG, "n_iters must be >= 0");
  return PASD_OK;
}

// Enqueue n_iters iterations of every context on `s`: contexts are grouped by
// (precision, order) and every group runs the kernels of an iteration as
// grouped launches over up to kMaxBatch problems.
void enqueue_batch(pasd_ctx* const* ctxs, int count, int n_iters, hipStream_t s) {
  std::vector<char> taken(count, 0);
  for (int i = 0; i < count; ++i) {
    if (taken[i]) continue;
    const int prec = ctxs[i]->cfg.precision, N = ctxs[i]->N;
    std::vector<pasd_ctx*> grp;
    for (int j = i; j < count; ++j)
      if (!taken[j] && ctxs[j]->cfg.precision == prec && ctxs[j]->N == N) {
        taken[j] = 1;
        grp.push_back(ctxs[j]);
      }
    for (size_t c0 = 0; c0 < grp.size(); c0 += kMaxBatch) {
      const int cnt = (int)std::min<size_t>(kMaxBatch, grp.size() - c0);
      if (prec == PASD_FP64) {
        LaunchSet<double> ls;
        ls.count = cnt;
        for (int r = 0; r < cnt; ++r) {
          ls.host[r] = &grp[c0 + r]->pd;
          ls.dev[r] = static_cast<const Problem<double>*>(grp[c0 + r]->dev_prob);
        }
        enqueue_iterations<double>(ls, n_iters, s, nullptr);
      } else {
        LaunchSet<float> ls;
        ls.count = cnt;
        for (int r = 0; r < cnt; ++r) {
          ls.host[r] = &grp[c0 + r]->pf;
          ls.dev[r] = static_cast<const Problem<float>*>(grp[c0 + r]->dev_prob);
        }
        enqueue_iterations<float>(ls, n_iters, s, nullptr);
      }
    }
  }
}

}  // namespace

// A captured batched step: n_iters iterations of a fixed set of contexts,
// replayed as one graph on the contexts' stream.
struct pasd_batch {
  std::vector<pasd_ctx*> ctxs;
  int dev = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

int pasd_step_batch(pasd_ctx* const* ctxs, int count, int n_iters) {
  g_last_error.clear();
  int rc = check_batch(ctxs, count, n_iters);
  if (rc != PASD_OK) return rc;
  if (count == 0 || n_iters == 0) return PASD_OK;
  DeviceGuard guard(ctxs[0]->dev);
  for (int i = 0; i < count; ++i) refresh_merged(ctxs[i], ctxs[i]->stream);
  enqueue_batch(ctxs, count, n_iters, ctxs[0]->stream);
  HIP_TRY(hipGetLastError());
  return PASD_OK;
}

void pasd_batch_destroy(pasd_batch* b) {
  if (!b) return;
  {
    DeviceGuard guard(b->dev);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  }
  delete b;
}

int pasd_batch_create(pasd_ctx* const* ctxs, int count, int n_iters, pasd_batch** out) {
  g_last_error.clear();
  if (!out) return fail(PASD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_batch(ctxs, count, n_iters);
  if (rc != PASD_OK) return rc;
  if (count == 0 || n_iters < 1) return fail(PASD_ERR_INVALID_ARG, "empty batch");
  DeviceGuard guard(ctxs[0]->dev);
  for (int i = 0; i < count; ++i) refresh_merged(ctxs[i], ctxs[i]->stream);
  pasd_batch* b = new pasd_batch();
  b->ctxs.assign(ctxs, ctxs + count);
  b->dev = ctxs[0]->dev;
  b->stream = ctxs[0]->stream;
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    b->cap_stream = nullptr;
    pasd_batch_destroy(b);
    return fail(PASD_ERR_HIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  }
  e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  hipGraph_t g = nullptr;
  if (e == hipSuccess) {
    enqueue_batch(ctxs, count, n_iters, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &g);
  }
  if (e == hipSuccess && g) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess || !b->exec) {
    (void)hipGetLastError();
    pasd_batch_destroy(b);
    return fail(PASD_ERR_HIP, std::string("capturing the batched step: ") + hipGetErrorString(e));
  }
  *out = b;
  return PASD_OK;
}

int pasd_batch_step(pasd_batch* b) {
  g_last_error.clear();
  if (!b || !b->exec) return fail(PASD_ERR_INVALID_ARG, "batch is NULL");
  DeviceGuard guard(b->dev);
  for (pasd_ctx* c : b->ctxs) refresh_merged(c, b->stream);
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  return PASD_OK;
}

int pasd_query_batch(pasd_ctx* const* ctxs, int count, pasd_info* infos) {
  g_last_error.clear();
  if (count < 0 || (count > 0 && (!ctxs || !infos))) return fail(PASD_ERR_INVALID_ARG, "bad arguments");
  std::vector<hipStream_t> streams;
  for (int i = 0; i < count; ++i) {
    pasd_ctx* ctx = ctxs[i];
    if (!ctx) return fail(PASD_ERR_INVALID_ARG, "NULL context");
    DeviceGuard guard(ctx->dev);
    DevScalars* dsc = ctx->cfg.precision == PASD_FP64 ? ctx->pd.sc : ctx->pf.sc;
    HIP_TRY(hipMemcpyAsync(ctx->host_sc, dsc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
    if (std::find(streams.begin(), streams.end(), ctx->stream) == streams.end())
      streams.push_back(ctx->stream);
  }
  for (hipStream_t s : streams) HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) fill_info(ctxs[i], &infos[i]);
  return PASD_OK;
}

int pasd_profile(pasd_ctx* ctx, int n_iters, double* ms, int* launches) {
  g_last_error.clear();
  if (!ctx || !ms) return fail(PASD_ERR_INVALID_ARG, "ctx or ms is NULL");
  if (n_iters < 1 || n_iters > 100000) return fail(PASD_ERR_INVALID_ARG, "n_iters out of range");
  DeviceGuard guard(ctx->dev);
  for (int k = 0; k < PASD_NUM_KERNELS; ++k) {
    ms[k] = 0;
    if (launches) launches[k] = 0;
  }
  const size_t nev = (size_t)n_iters * PASD_NUM_KERNELS + 1;
  std::vector<hipEvent_t> ev(nev, nullptr);
  int rc = PASD_OK;
  size_t made = 0;
  for (; made < nev; ++made) {
    hipError_t e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) {
      rc = fail(PASD_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
      break;
    }
  }
  if (rc == PASD_OK) rc = enqueue(ctx, n_iters, ev.data());
  if (rc == PASD_OK) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = fail(PASD_ERR_HIP, std::string("profile: ") + hipGetErrorString(e));
  }
  if (rc == PASD_OK) {
    for (int it = 0; it < n_iters; ++it)
      for (int k = 0; k < PASD_NUM_KERNELS; ++k) {
        const size_t i = (size_t)it * PASD_NUM_KERNELS + k;
        float t = 0;
        if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) == hipSuccess) ms[k] += t;
        if (launches) launches[k] += 1;
      }
  }
  for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Solve without allocation (pasd_solve_static).  The whole solver state of one
// solve (D, Y_n, the factors, the split-K partials of the GEMM-M reduction and
// of the Gram, the control scalars and the problem descriptors) lives in one
// file-scope device array of kStaticScratchBytes per GPU, which the code
// object holds from load until the process ends.  Host code never passes the
// array's name to a kernel or a copy: its device address is resolved once per
// device with hipGetSymbolAddress (with that device current) and kept in
// g_scratch_dev.  Every call on a device reuses that device's array: the
// state is cleared by a fill kernel at the start of each call, and calls that
// overlap on one device race on it.
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kStaticScratchBytes = size_t(32) << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` on each device, once resolved

// Device address of `scratch` on device `dev` (the current device).
int static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PASD_ERR_UNSUPPORTED, "pasd_solve_static: device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PASD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return PASD_OK;
}

}  // namespace

extern "C" {

size_t pasd_static_scratch_bytes(void) { return kStaticScratchBytes; }

int pasd_solve_static(const pasd_config* cfg, const void* T, void* X, void* E, pasd_info* info) {
  g_last_error.clear();
  int rc = validate_impl(cfg);
  if (rc != PASD_OK) return rc;
  if (!T) return fail(PASD_ERR_INVALID_ARG, "T is NULL");
  Plan pl;
  make_plan(cfg, pl, /*own_T=*/false);  // T is read in place from the caller's buffer
  if (pl.L.total > kStaticScratchBytes)
    return fail(PASD_ERR_UNSUPPORTED, "pasd_solve_static: the solve needs " +
                                          std::to_string(pl.L.total) + " bytes of state, above the " +
                                          std::to_string(kStaticScratchBytes) + "-byte static scratch");
  pasd_ctx ctx;  // host descriptor only; nothing of it is allocated
  rc = ctx_init_host(&ctx, cfg, pl);
  if (rc != PASD_OK) return rc;
  ctx.graph_disabled = true;  // direct launches: instantiating a graph would allocate
  DeviceGuard guard(ctx.dev);
  void* base = nullptr;
  rc = static_scratch(ctx.dev, &base);
  if (rc != PASD_OK) return rc;
  DevScalars host_sc;
  ctx.host_sc = &host_sc;
  ctx.bytes = pl.L.total;
  rc = ctx_init_device(&ctx, pl, base, T, /*T_on_device=*/1, /*T_in_place=*/true);
  const int status = rc == PASD_OK ? pasd_solve(&ctx, info) : rc;
  if (status < 0) {
    (void)hipStreamSynchronize(ctx.stream);
    return status;
  }
  if (X || E) {
    rc = pasd_get_result(&ctx, X, E, /*on_device=*/1);
    if (rc != PASD_OK) return rc;
  }
  return status;
}

void pasd_destroy(pasd_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard guard(ctx->dev);
    if (ctx->base || ctx->scratch_out) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->base) (void)hipFree(ctx->base);
    if (ctx->scratch_out) (void)hipFree(ctx->scratch_out);
    if (ctx->host_sc) (void)hipHostFree(ctx->host_sc);
    if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  }
  delete ctx;
}

const char* pasd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
