// Internal declarations shared by the PASD HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pasd.h"

namespace pasd {

constexpr int kMaxN = PASD_MAX_ORDER;
constexpr int kRT = 16;        // rank tile: R_n is padded to 16 in the factors and partials
constexpr int kResSlots = 64;  // residual maxima are spread over this many words per mode

// Geometry of the mode-n unfolding of a row-major tensor viewed as (A, I, B):
// element (a, i, b) sits at a*I*B + i*B + b, column index j = a*B + b.
struct ModeGeom {
  int64_t A, B, J;  // J = A*B
  int I, R;
};

// Device-resident control state of one context.
struct DevScalars {
  double mu;
  int k;
  int done;  // 0 running, 1 converged, 2 max_iter, 3 numeric
  int converged;
  int pad;
  double residual[kMaxN];              // residuals of the last completed iteration
  int rank[kMaxN];
  int eig_sweeps[kMaxN];               // Jacobi sweeps of the last eigensolve
  // per-iteration residual maxima as double bits, block b of the fused pass
  // updates slot b % kResSlots with atomicMax; the control kernel folds them
  unsigned long long res_slots[kMaxN][kResSlots];
};

// Per-mode device pointers (state type S for P and Uf, double for U/M/S).
template <typename S>
struct ModeBufs {
  S* Y;          // multiplier, numel
  S* P;          // R x J (row-major)
  double* U;     // I x R (row-major)  active subspace
  S* Us;         // I x kRT  U in the state type, zero-padded columns (GEMM-P operand)
  S* Uf;         // I x kRT  U W (SVT-folded factor), padded rows of 16
  S* UfT;        // kRT x I  transposed copy (last mode uses it)
  double* Mpart; // GEMM-M split-K partials [nblk][I][kRT] (double)
  double* M;     // reduced M, I x kRT
  double* Spart; // Gram partials [nblk][kRT][kRT]
  double* Wf;    // kRT x kRT SVT factor
  double* Wev;   // kRT x kRT eigenvectors of the last Gram (warm start)
  int mblocks;   // number of GEMM-M partial blocks
  int sblocks;   // number of Gram partial blocks
};

// Everything a kernel needs about the problem, passed by value.
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
  double* hist;  // residual history [max_iter][N]
};

// Launchers (each enqueues on `stream`; kernels read sc->done and skip).
template <typename S> void launch_gemm_m(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_reduce_m(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_qr(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_gemm_p(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_gram(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_eig(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_fused(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_control(const Problem<S>& p, hipStream_t s);
template <typename S> void launch_init(const Problem<S>& p, double mu0, hipStream_t s);
template <typename S> void launch_output(const Problem<S>& p, S* X, S* E, hipStream_t s);
template <typename S> void launch_component(const Problem<S>& p, int n, S* Z, hipStream_t s);

// Block counts chosen on the host for the split-K kernels.
int gemm_m_blocks(const ModeGeom& g);
int gram_blocks(const ModeGeom& g);

}  // namespace pasd
