// Internal declarations shared by the PASD HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pasd.h"

namespace pasd {

constexpr int kMaxN = PASD_MAX_ORDER;
constexpr int kRT = 16;        // rank tile: R_n is padded to 16 in the factors and partials
constexpr int kMaxTiles = PASD_MAX_RANK / kRT;  // rank tiles of the widest mode
constexpr int kResSlots = 64;  // residual maxima are spread over this many words per mode
constexpr int kXcds = 8;       // accelerator complex dies of gfx950; blocks are dealt to them in turn
constexpr int kCUs = 256;      // compute units of the MI355X

// Division by a divisor d >= 1 fixed for a whole launch, by multiply-high,
// add and shift (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, the round-up method): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, n / d = (umulhi(n, m) + n) >> l for
// 0 <= n < 2^32; kernels use it for n < 2^31, where the sum cannot overflow.
struct FastDiv {
  uint32_t m, l;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
  return FastDiv{(uint32_t)m, l};
}
__host__ __device__ inline uint32_t fastdiv(uint32_t n, FastDiv f) {
  const uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
  return (hi + n) >> f.l;
}

// Geometry of the mode-n unfolding of a row-major tensor viewed as (A, I, B):
// element (a, i, b) sits at a*I*B + i*B + b, column index j = a*B + b.
struct ModeGeom {
  int64_t A, B, J;  // J = A*B
  int I, R;
  int T;  // rank tiles, ceil(R / kRT); the factors are padded to T * kRT columns
};

// Device-resident control state of one context.
struct DevScalars {
  double mu;
  int k;
  int done;  // 0 running, 1 converged, 2 max_iter, 3 numeric, 4 precision floor
  int converged;
  int pad;
  double residual[kMaxN];              // residuals of the last completed iteration
  int rank[kMaxN];
  int eig_sweeps[kMaxN];               // Jacobi sweeps of the last eigensolve
  double dmax;                         // max |D| of the last iteration
  double tol_eff;                      // tolerance the last stopping test used
  // per-iteration residual maxima as double bits, block b of the fused pass
  // updates slot b % kResSlots with atomicMax; the control kernel folds them
  // (row kMaxN holds max |D|)
  unsigned long long res_slots[kMaxN + 1][kResSlots];
};

// Per-mode device pointers (state type S for P and Uf, double for U/M/S).
template <typename S>
struct ModeBufs {
  S* Y;          // multiplier, numel
  // Rank-indexed factors with R > kRT are stored tile-major: T blocks, block t
  // holding columns kRT t .. kRT t + kRT - 1 in the one-tile layout, so that a
  // tile is itself a valid one-tile factor.  RT = T kRT below.
  S* P;          // RT x J (row-major; rows >= R zero)
  double* U;     // I x R (row-major)  active subspace
  S* Us;         // [T][I][kRT]  U in the state type, zero-padded columns (GEMM-P operand)
  S* Uf;         // [T][I][kRT]  U W (SVT-folded factor)
  S* UfT;        // RT x I  transposed copy (last mode uses it)
  double* Mpart; // GEMM-M split-K partials [T][nblk][I][R_t] (double), R_t = min(R - kRT t, kRT)
  double* M;     // reduced M, [T][I][kRT] (columns >= R unused)
  double* Spart; // Gram partials [nblk][RT][RT]
  double* Wf;    // RT x RT SVT factor
  double* Wev;   // RT x RT eigenvectors of the last Gram (warm start)
  double* Fac;   // RT SVT weights f_i of the last eigensolve (f_i > 0: V_n keeps direction i)
  double* Mf;    // merged modes: the fused pass's partials of the next M_n, [fused_blocks][kRT]
  double* Mq;    // fast modes folded into the fused pass (Problem::mfull): its per-block
                 // partials of the next M_n, [fused_blocks][I][R]
  unsigned int* mcnt;  // with Mq: per 64-entry tile of M_n, the k_msum blocks done (0 between launches)
  int mblocks;   // number of GEMM-M partial blocks
  int sblocks;   // number of Gram partial blocks
};

// Kernels with a per-mode grid: index into Problem::kb.
enum ModeKernel { KB_GEMM_M = 0, KB_REDUCE_M, KB_GEMM_P, KB_GRAM, KB_MSUM, KB_COUNT };

// Groups of fused blocks whose fast-mode partials k_msum sums first; k_reduce_m
// then adds the group sums (Problem::mfull).
constexpr int kMsumGroups = 64;

// Everything a kernel needs about one solve.  A device copy lives in the
// solve's own allocation; kernels reach it through a pointer in Batch.
template <typename S>
struct Problem {
  int N;
  int64_t numel;
  ModeGeom g[kMaxN];
  ModeBufs<S> m[kMaxN];
  const S* T;
  S* D;  // D = T - E
  DevScalars* sc;
  double lam[kMaxN];
  double alpha[kMaxN];
  double mu_max, rho, tol;
  int max_iter;
  int precision;
  int tiebreak_keep;  // PASD_FLAG_TIEBREAK_KEEP
  int floor_stop;     // stop at the precision floor (PASD_FLAG_NO_FLOOR_STOP clear)
  double* hist;  // residual history [max_iter][N]
  // first block of every mode within this problem's grid, per kernel kind
  int kb[KB_COUNT][kMaxN + 1];
  int fused_blocks;  // blocks of the fused pass for this problem
  int vecw;          // last dimension divisible by the 16-byte vector width (fused pass)
  int idx32;         // every element offset of the fused pass fits 32-bit byte offsets
  // Order of the fused pass over the 8 XCDs.  0: XCD x sweeps the x-th
  // contiguous eighth of the tensor.  1 (chosen when P_0 is too large to stay
  // in one XCD's L2, N >= 3, I_1 divisible by 8, 32-bit offsets): XCD x
  // sweeps, for every mode-0 index in turn, the x-th eighth of the mode-1
  // range, so that it only needs the eighth of P_0's columns with i_1 in that
  // range.  In chunks of the pass: f_cp0 per mode-0 slab, f_cp1 per mode-1
  // slab, f_seg = f_cp1 I_1 / 8 per segment (one mode-0 index, one XCD).
  int fsplit1;
  uint32_t f_cp0, f_cp1, f_seg;
  FastDiv fd_seg;
  // GEMM-M of the next iteration folded into the fused pass for the modes
  // 0 .. mmerge-1 (mmerge > 0): the pass runs fused_blocks blocks, block b over
  // the mcb consecutive chunks from b mcb on, a range inside one mode-n slab
  // (B_n consecutive elements, one index i_n) for every merged mode; each
  // block writes its partial sums of M_n[i_n, :] = sum G_n(x) P_n[:, j_n(x)]
  // over its range to ModeBufs::Mf, and the GEMM-M reduction adds the
  // mslab[n] blocks of every slab with index i_n.  GEMM-M has no blocks for
  // these modes.
  int mmerge;
  uint32_t mcb;
  int mslab[kMaxN];
  // mfull (order 4, FP64 state, merged modes 0 and 1): the fused pass also
  // accumulates the next M_n of the fast modes 2 and 3.  Every chunk of a
  // thread then has the same last-mode columns i_3 .. i_3 + vec - 1 (the row
  // length in chunks, Q, divides 256 and mcb, Q <= 64), so the thread keeps
  // FP64 sums of G_3(x) P_3[:, j_3(x)] for its columns, and a row (one i_2,
  // Q aligned lanes) sums G_2(x) P_2[:, j_2(x)] across its lanes; each block
  // writes I_n x R partials to ModeBufs::Mq, k_msum adds them in kMsumGroups
  // groups of consecutive blocks (in block order) to ModeBufs::Mpart and the
  // last of a tile's blocks adds the groups into M_n; k_msum also reduces the
  // merged modes' slab sums.  Neither GEMM-M nor k_reduce_m runs for such a
  // problem.
  int mfull;
  // GEMM-P blocks of the last two modes taken together (k_gemm_p2; every
  // R_n <= kRT, I_{N-2} = I_{N-1} = 64, N >= 3): one per 64 x 64 slab, 0
  // otherwise; those modes then have no blocks of their own in kb[KB_GEMM_P]
  int gp2;
  // The fused pass writes D and Y_n with non-temporal stores: together they
  // exceed the 256 MB Infinity Cache ((N + 1) L s > 256 MiB), so no later
  // kernel finds them there, and allocating them in the caches only evicts the
  // factor columns the pass re-reads (64^4 FP64: 0.588 -> 0.584 ms per
  // iteration; at 200^3 FP32, 128 MB, GEMM-M rereads them from the Infinity
  // Cache and non-temporal stores cost it 5 us).
  int ntstore;
  // fused pass divisors: chunks per row of the last mode, and per mode n < N-1
  // the rows per mode-n fibre index (B_n / I_N) and I_n
  FastDiv fd_q;
  FastDiv fd_rb[kMaxN];
  FastDiv fd_i[kMaxN];
  // unfolding GEMMs: B_n, for column indices j < 2^31
  FastDiv fd_b[kMaxN];
  // Some R_n > kRT: the rank-wide kernels run this problem.  The unfolding
  // GEMMs and the GEMM-M reduction, which work on one rank tile, run it as
  // `ntiles` views: view t is a copy whose mode n carries tile t alone (R_n
  // replaced by R_t, the tile's factor pointers, no blocks where kRT t >= R_n).
  // Host code only reads the view pointers.
  int wide;
  int ntiles;
  const Problem* view_host[kMaxTiles];
  const Problem* view_dev[kMaxTiles];
};

// One launch over up to kMaxBatch problems (kernel arguments, ~1.6 KB): block
// b belongs to problem r with start[r] <= b < start[r + 1].  A single solve
// is a batch of one; a serving step batches every resident solve.
constexpr int kMaxBatch = 128;
template <typename S>
struct Batch {
  const Problem<S>* p[kMaxBatch];
  int start[kMaxBatch + 1];
  int nreq;
};

__device__ __forceinline__ int batch_find(const int* start, int nreq, int blk) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk >= start[mid]) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Blocks of a launch are dealt to the XCDs in turn (global block g to XCD
// g mod kXcds).  For the nt consecutive blocks m0 .. m0 + nt - 1 of one work
// range, return the position of local block b in an order that lists each
// XCD's blocks contiguously (XCD 0's first, ...): consecutive positions then
// run on one XCD and share its L2.  A bijection on [0, nt) for any nt, m0.
__host__ __device__ inline int xcd_order(int b, int nt, int m0) {
  const int first_cls = m0 % kXcds;  // class of local block 0
  const int c = (first_cls + b) % kXcds;
  int off = 0;
  for (int y = 0; y < c; ++y) {
    const int f = (y - first_cls + kXcds) % kXcds;  // first local block of class y
    off += f < nt ? (nt - f + kXcds - 1) / kXcds : 0;
  }
  const int f = (c - first_cls + kXcds) % kXcds;
  return off + (b - f) / kXcds;
}

__device__ __forceinline__ int mode_of(const int* kb, int N, int lblk) {
  int n = 0;
  while (n + 1 < N && lblk >= kb[n + 1]) ++n;
  return n;
}

// Host view of a launch: host copies (for grid sizes and template choices)
// and device copies (what the kernels dereference) of the same problems.
// A double moved across lanes by a DPP control (within rows of 16 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror, row_mirror
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <typename S>
struct LaunchSet {
  int count = 0;
  const Problem<S>* host[kMaxBatch];
  const Problem<S>* dev[kMaxBatch];
};

template <typename S>
inline bool any_wide(const LaunchSet<S>& ls) {
  for (int r = 0; r < ls.count; ++r)
    if (ls.host[r]->wide) return true;
  return false;
}

// Problems of a set with every R_n <= kRT, and those with some R_n > kRT.
template <typename S>
inline void split_wide(const LaunchSet<S>& ls, LaunchSet<S>& narrow, LaunchSet<S>& wide) {
  narrow.count = 0;
  wide.count = 0;
  for (int r = 0; r < ls.count; ++r) {
    LaunchSet<S>& d = ls.host[r]->wide ? wide : narrow;
    d.host[d.count] = ls.host[r];
    d.dev[d.count] = ls.dev[r];
    ++d.count;
  }
}

// Launchers of one iteration's kernels over a set (each enqueues on `s`;
// kernels read sc->done of their problem and skip).
template <typename S> void launch_gemm_m(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_reduce_m(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_qr(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_gemm_p(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_gram(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_eig(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_fused(const LaunchSet<S>& ls, hipStream_t s);
template <typename S> void launch_control(const LaunchSet<S>& ls, hipStream_t s);
// Single-problem utilities.
template <typename S> void launch_init(const Problem<S>& p, double mu0, hipStream_t s);
template <typename S> void launch_output(const Problem<S>& p, S* X, S* E, hipStream_t s);
template <typename S> void launch_component(const Problem<S>& p, int n, S* Z, hipStream_t s);
// Recompute the merged modes' GEMM-M partials from the stored state (after a
// checkpoint import), with the fused pass's own arithmetic and order.
template <typename S> void launch_mrefresh(const LaunchSet<S>& ls, hipStream_t s);

// Modes whose GEMM-M folds into the fused pass (see Problem::mmerge): for a
// tensor of order N with last-mode vector width vec and nchunk = numel / vec
// chunks, sets *mmerge (0: none), *mcb (chunks per fused block) and *blocks.
void merge_plan(const int64_t* dims, int N, int64_t numel, int vec, int max_rank, int state_bytes,
                bool idx32, int* mmerge, int64_t* mcb, int* blocks, int* mfull);

// Grid sizes chosen on the host.
int gemm_m_blocks(const ModeGeom& g, int N);
int msum_blocks(const ModeGeom& g);
int gram_blocks(const ModeGeom& g);
int gemm_p_blocks(const ModeGeom& g);
int reduce_m_blocks(const ModeGeom& g);
int fused_blocks(int64_t numel, int vec);

// Fill a Batch from a set, with `blocks(problem)` blocks per problem.
template <typename S, typename F>
inline int make_batch(const LaunchSet<S>& ls, Batch<S>& b, F blocks) {
  int tot = 0;
  b.nreq = ls.count;
  for (int r = 0; r < ls.count; ++r) {
    b.p[r] = ls.dev[r];
    b.start[r] = tot;
    tot += blocks(*ls.host[r]);
  }
  b.start[ls.count] = tot;
  return tot;
}

}  // namespace pasd
