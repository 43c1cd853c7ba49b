// Small per-mode FP64 kernels of the PASD iteration, one block per (problem, mode).
//
//   k_qr* : U_n = an orthonormal basis of range(M_n), M_n = G_n P_n^T, which is
//           the range of the Procrustes solution of eqs. (9)-(10); the iterates
//           depend on range(U_n) only, so any orthonormal basis of it will do.
//           CholeskyQR2 on the matrix cores where M_n is well conditioned,
//           Householder QR otherwise (it stays orthonormal when M_n is rank
//           deficient).
//   k_eig : S_n = P_n P_n^T = W diag(l) W^T by parallel cyclic Jacobi; with
//           s_i = sqrt(l_i) (the singular values of P_n) and tau = lambda_n / mu,
//           SVT_tau(P_n) = W diag((s_i - tau)_+ / s_i) W^T P_n (eq. (13)); the
//           kernel stores the R x R factor W_f = W diag(f) W^T and U_n W_f, so
//           that Z_n = fold_n(U_n W_f P_n) is formed later without V_n.
#include <math.h>

#include "pasd_internal.hpp"

namespace pasd {

constexpr int kQrLds = 8192;  // doubles of LDS for M (I_n * R_n <= 8192)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename S>
__global__ void __launch_bounds__(64) k_qr(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, lane = threadIdx.x;
  __shared__ double A[kQrLds];  // column-major A[c * I + i]
  __shared__ double tau[kRT];
  for (int e = lane; e < I * R; e += 64) {
    const int i = e / R, c = e - i * R;
    A[c * I + i] = mb.M[(int64_t)i * kRT + c];
  }
  __syncthreads();
  // Householder QR (LAPACK dgeqr2 convention: v = (1, v_tail), H = I - t v v^T).
  for (int c = 0; c < R; ++c) {
    double part = 0;
    for (int i = c + 1 + lane; i < I; i += 64) {
      const double x = A[c * I + i];
      part += x * x;
    }
    const double xnorm2 = wave_sum(part);
    const double alpha = A[c * I + c];
    double t = 0, beta = alpha, scale = 0;
    if (xnorm2 > 0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (xnorm2 > 0)
      for (int i = c + 1 + lane; i < I; i += 64) A[c * I + i] *= scale;
    __syncthreads();
    // w_j = v^T A[c:, j] for all j > c, then A[c:, j] -= t w_j v
    double w[kRT];
#pragma unroll
    for (int jj = 0; jj < kRT; ++jj) w[jj] = 0;
    for (int i = c + 1 + lane; i < I; i += 64) {
      const double v = A[c * I + i];
#pragma unroll
      for (int jj = 0; jj < kRT; ++jj)
        if (c + 1 + jj < R) w[jj] += v * A[(c + 1 + jj) * I + i];
    }
#pragma unroll
    for (int jj = 0; jj < kRT; ++jj)
      if (c + 1 + jj < R) w[jj] = wave_sum(w[jj]) + A[(c + 1 + jj) * I + c];
    __syncthreads();
    if (t != 0) {
      for (int i = c + 1 + lane; i < I; i += 64) {
        const double v = A[c * I + i];
#pragma unroll
        for (int jj = 0; jj < kRT; ++jj)
          if (c + 1 + jj < R) A[(c + 1 + jj) * I + i] -= t * w[jj] * v;
      }
      if (lane == 0) {
#pragma unroll
        for (int jj = 0; jj < kRT; ++jj)
          if (c + 1 + jj < R) A[(c + 1 + jj) * I + c] -= t * w[jj];
      }
    }
    if (lane == 0) {
      A[c * I + c] = beta;
      tau[c] = t;
    }
    __syncthreads();
  }
  // Accumulate Q = H_0 H_1 ... H_{R-1} [I_R; 0] in place (LAPACK dorg2r order).
  for (int c = R - 1; c >= 0; --c) {
    const double t = tau[c];
    double w[kRT];
#pragma unroll
    for (int jj = 0; jj < kRT; ++jj) w[jj] = 0;
    for (int i = c + 1 + lane; i < I; i += 64) {
      const double v = A[c * I + i];
#pragma unroll
      for (int jj = 0; jj < kRT; ++jj)
        if (c + 1 + jj < R) w[jj] += v * A[(c + 1 + jj) * I + i];
    }
#pragma unroll
    for (int jj = 0; jj < kRT; ++jj)
      if (c + 1 + jj < R) w[jj] = wave_sum(w[jj]) + A[(c + 1 + jj) * I + c];
    __syncthreads();
    for (int i = c + 1 + lane; i < I; i += 64) {
      const double v = A[c * I + i];
#pragma unroll
      for (int jj = 0; jj < kRT; ++jj)
        if (c + 1 + jj < R) A[(c + 1 + jj) * I + i] -= t * w[jj] * v;
      A[c * I + i] = -t * v;
    }
    if (lane == 0) {
#pragma unroll
      for (int jj = 0; jj < kRT; ++jj)
        if (c + 1 + jj < R) A[(c + 1 + jj) * I + c] -= t * w[jj];
      A[c * I + c] = 1.0 - t;
    }
    for (int i = lane; i < c; i += 64) A[c * I + i] = 0.0;
    __syncthreads();
  }
  for (int e = lane; e < I * kRT; e += 64) {
    const int i = e / kRT, c = e - i * kRT;
    const double v = c < R ? A[c * I + i] : 0.0;
    if (c < R) mb.U[(int64_t)i * R + c] = v;
    mb.Us[e] = (S)v;
  }
}

// ---------------------------------------------------------------------------
// SVT factor by a warm-started parallel cyclic Jacobi on the R x R Gram, one
// 256-thread block per (problem, mode):
//  1. S = sum of the Gram partials (one entry per thread, all partials loaded
//     at once) while U_n is staged in LDS;
//  2. S' = W0^T S W0 with W0 the eigenvectors of the previous iteration
//     (identity at k = 0), so that S' is nearly diagonal once the iteration
//     settles; the eigenvectors are accumulated as W = W0 J_1 J_2 ...;
//  3. before each sweep the block checks whether any pair still needs a
//     rotation, so a converged matrix costs one check instead of a sweep;
//  4. round-robin Jacobi: every round rotates R'/2 disjoint pairs (R' = R
//     rounded up to even, a dummy index for odd R); each thread recomputes
//     the rotations of the pairs it touches (jacobi_rotation, branch-free),
//     issues all of its reads first, reads the matrix from one buffer and
//     writes the other, so a round has one barrier;
//  5. W_f = W diag(f) W^T and U W_f (FP64 MFMA).
// A pair is rotated while |s_pq| > thr sqrt(|s_pp s_qq|) (and |s_pq| > 1e-150,
// see jacobi_needed), thr = 4e-16 for an FP64 state and 2^-24 for FP32.  Why
// that suffices: W_f = F(S) with F(l) = (1 - tau / sqrt(l))_+ on the
// eigenvalues, and a remaining off-diagonal entry e of the rotated S moves
// W_f by about |e| times the divided difference (F(l_p) - F(l_q)) / (l_p - l_q),
// which is at most 1 / (2 sqrt(l_p l_q)) (with x = sqrt(l_p) > y = sqrt(l_q)
// >= tau it equals tau / (x y (x + y)); below tau^2 F is zero); so with
// |e| <= thr sqrt(l_p l_q) W_f moves by at most thr / 2, under the rounding of
// the FP32 factors U W_f.
// W_f is a spectral function of S, so it does not depend on W0 beyond rounding.
// ---------------------------------------------------------------------------
constexpr int kEigParts = 64;  // Gram partials (at most; see gram_blocks), loaded in one pass

// Pair idx of round rd of the round-robin (chess tournament) ordering of the
// indices 0 .. m (m odd): index m stays, the others rotate; p < q.
__device__ __forceinline__ void rr_pair(int rd, int idx, int m, int& p, int& q) {
  if (idx == 0) {
    p = m;
    q = rd;
  } else {  // (rd + idx) mod m and (rd - idx) mod m; both operands lie in [0, 2m)
    p = rd + idx;
    p = p >= m ? p - m : p;
    q = rd - idx + m;
    q = q >= m ? q - m : q;
  }
  if (p > q) {
    const int tmp = p;
    p = q;
    q = tmp;
  }
}

// The round of the round-robin ordering (rr_pair, indices 0 .. m, m odd) in
// which pair p < q is rotated: round p when q is the fixed index m, else the
// round rd with p + q = 2 rd (mod m), i.e. rd = (p + q) (m + 1) / 2 mod m.
__device__ __forceinline__ int rr_round(int p, int q, int m) {
  return q == m ? p : (int)(((unsigned)(p + q) * (unsigned)((m + 1) / 2)) % (unsigned)m);
}

// 1/sqrt(a) and 1/a for normal a > 0: the hardware estimates (v_rsq_f64,
// v_rcp_f64, relative error near 2^-23) refined by two Newton steps each,
// h <- h + h (1 - a h^2) / 2 and r <- r + r (1 - a r), which square the error
// twice (to the rounding level).  Much shorter dependent chains than the
// correctly rounded library square root and division.
__device__ __forceinline__ double rsqrt_nr(double a) {
  double h = __builtin_amdgcn_rsq(a);
  h = fma(0.5 * h, fma(-a * h, h, 1.0), h);
  h = fma(0.5 * h, fma(-a * h, h, 1.0), h);
  return h;
}
__device__ __forceinline__ double rcp_nr(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(fma(-a, r, 1.0), r, r);
  r = fma(fma(-a, r, 1.0), r, r);
  return r;
}

// Whether the pair (p, q) of the symmetric A needs a rotation:
// |a_pq| > thr sqrt(|a_pp a_qq|), compared in squares, and |a_pq| > 1e-150 so
// that the squares below stay normal.  (A matrix below that scale has every
// singular value far under the threshold tau: its SVT factor is zero.)
template <int LD>
__device__ __forceinline__ bool jacobi_needed(const double (*A)[LD], int p, int q, double thr) {
  const double b = fabs(A[p][q]);
  return b > 1e-150 && b * b > thr * thr * fabs(A[p][p]) * fabs(A[q][q]);
}

// Pairs whose 2 x 2 block lies wholly below the SVT threshold tau^2 on the
// eigenvalues of S: both diagonal entries below t2h = tau^2 / 2 and the
// coupling below t2r = tau^2 / (2 R).  They are not rotated.  W_f = F(S) with
// F = 0 below tau^2, so a rotation inside that part cannot change W_f; once
// every other pair has converged, the indices with diagonal below tau^2 / 2
// span an invariant subspace whose eigenvalues are below tau^2 / 2 +
// (R - 1) tau^2 / (2 R) < tau^2 (Gershgorin on that block), where f = 0 is
// exact, and f_i computed from those diagonal entries is 0 as well.  This
// saves the sweeps that would otherwise diagonalise directions the SVT
// discards (the surplus R_n - r, and most directions while mu is small).
__device__ __forceinline__ bool jacobi_discarded(double a, double d, double b, double t2h,
                                                 double t2r) {
  return a < t2h && d < t2h && fabs(b) < t2r;
}

// Rotation (c, s, t = s / c) that annihilates the off-diagonal b of the
// symmetric 2x2 block [[a, b], [b, d]], in Rutishauser's form:
// x = d - a, y = 2 b, r = hypot(x, y), w = |x| + r, c = w / hypot(w, y),
// s = sgn(x) y / hypot(w, y), t = sgn(x) y / w.  The identity when !valid (the
// padding index) or below the threshold.  Branch-free (the result is selected
// at the end; a discarded lane may compute with infinities), so that the loads
// and the arithmetic of several rotations overlap.
__device__ __forceinline__ void jacobi_rotation(double a, double d, double b, bool valid, double thr,
                                                double& c, double& s, double& t) {
  const double ab = fabs(b);
  const bool need = valid && ab > 1e-150 && ab * ab > thr * thr * fabs(a) * fabs(d);
  const double x = d - a, y = 2.0 * b;
  const double n1 = fma(x, x, y * y);
  const double r = n1 * rsqrt_nr(n1);
  const double w = fabs(x) + r;
  const double sy = x >= 0.0 ? y : -y;
  const double h = rsqrt_nr(fma(w, w, y * y));
  c = need ? w * h : 1.0;
  s = need ? sy * h : 0.0;
  t = need ? sy * rcp_nr(w) : 0.0;
}

template <typename S>
__global__ void __launch_bounds__(256) k_eig(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int R = g.R, I = g.I, tid = threadIdx.x;
  const bool warm = pb.sc->k > 0;
  __shared__ double Sb[2][kRT][kRT + 1];  // the Gram in two buffers (Jacobi rounds alternate)
  __shared__ double W[kRT][kRT + 1];
  __shared__ double T1[kRT][kRT + 1];
  __shared__ double fac[kRT];
  __shared__ unsigned int rmask[2];  // rounds of the coming sweep with a pair to rotate
  __shared__ double Ul[kQrLds];
  double (*Sm)[kRT + 1] = Sb[0];
  {
    const int r = tid / kRT, c = tid % kRT;
    const bool in = r < R && c < R;
    // all loads of this thread first: its share of U_n, then the partials
    // Loads are unconditional (indices clamped into range, values masked
    // afterwards): a load under a condition is compiled as a branch with a
    // wait after it, which serialises the round trips.
    constexpr int kU = 8;
    const int nU = I * R;
    double uv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = tid + 256 * u;
      uv[u] = mb.U[e < nU ? e : nU - 1];
    }
    const double wev = mb.Wev[tid];
    // every partial in one pass of loads (the Gram kernel writes at most
    // kEigParts of them), static register indices (no private memory)
    const int nb = mb.sblocks;
    const double* sp = mb.Spart + tid;
    double part[kEigParts];
#pragma unroll
    for (int b = 0; b < kEigParts; ++b) part[b] = sp[(int64_t)(b < nb ? b : nb - 1) * kRT * kRT];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int b = 0; b < kEigParts; ++b) part[b] = (in && b < nb) ? part[b] : 0.0;
    // fixed-order pairwise sum of the partials
#pragma unroll
    for (int w = kEigParts / 2; w > 0; w /= 2)
#pragma unroll
      for (int b = 0; b < w; ++b) part[b] += part[b + w];
    Sm[r][c] = part[0];
    W[r][c] = (warm && in) ? wev : (r == c ? 1.0 : 0.0);
    // U_n is staged in LDS when it fits (a tall mode reads it from global
    // memory below)
    if (nU <= kQrLds) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = tid + 256 * u;
        if (e < nU) Ul[e] = uv[u];
      }
      for (int e = tid + 256 * kU; e < nU; e += 256) Ul[e] = mb.U[e];
    }
  }
  __syncthreads();
  {  // T1 = S W0 with the upper triangle of S mirrored
    const int r = tid / kRT, c = tid % kRT;
    double t = 0;
    for (int k = 0; k < R; ++k) t += (r <= k ? Sm[r][k] : Sm[k][r]) * W[k][c];
    T1[r][c] = t;
  }
  __syncthreads();
  {  // S' = W0^T T1, upper triangle mirrored
    const int r = tid / kRT, c = tid % kRT;
    const int rr = r <= c ? r : c, cc = r <= c ? c : r;
    double v = 0;
    for (int k = 0; k < R; ++k) v += W[k][rr] * T1[k][cc];
    __syncthreads();
    Sm[r][c] = (r < R && c < R) ? v : 0.0;
  }
  __syncthreads();
  const double thr = sizeof(S) == 4 ? 5.9604644775390625e-08 : 4.0e-16;
  const double tau = pb.lam[n] / pb.sc->mu;
  const double t2h = 0.5 * tau * tau, t2r = t2h / R;
  const int Rp = R + (R & 1);
  const int half = Rp / 2;
  const int m = Rp - 1;
  int sweeps = 0;
  int cur = 0;  // Sb[cur] holds the current matrix
  if (tid < 2) rmask[tid] = 0u;
  __syncthreads();
  for (int sweep = 0; sweep < 40 && R > 1; ++sweep) {
    int need = 0;
    {
      const int p = tid / kRT, q = tid % kRT;
      if (p < q && q < R)
        need = jacobi_needed(Sb[cur], p, q, thr) &&
               !jacobi_discarded(Sb[cur][p][p], Sb[cur][q][q], Sb[cur][p][q], t2h, t2r);
      if (need) atomicOr(&rmask[sweep & 1], 1u << rr_round(p, q, m));
    }
    if (!__syncthreads_or(need)) break;
    sweeps = sweep + 1;
    // Rounds whose pairs all passed the check are skipped: a rotation in an
    // earlier round can push one of their pairs back over the threshold, and
    // the next check then starts another sweep, so the stopping criterion is
    // unchanged.
    const unsigned int mask = rmask[sweep & 1];
    if (tid == 0) rmask[(sweep + 1) & 1] = 0u;  // every thread read it before this sweep's check
    for (int rd = 0; rd < m; ++rd) {
      if (!((mask >> rd) & 1u)) continue;
      // Every thread derives the pairs and rotations it needs from the round
      // number and the current matrix, so a round is one read of Sb[cur], one
      // write of every entry of the other buffer, and one barrier.
      const double (*A)[kRT + 1] = Sb[cur];
      double (*B)[kRT + 1] = Sb[cur ^ 1];
      if (tid < half * half) {
        const int k = tid / half, l = tid - k * half;
        if (k <= l) {
          int pk, qk, pl, ql;
          rr_pair(rd, k, m, pk, qk);
          rr_pair(rd, l, m, pl, ql);
          // every read of the round first, then the arithmetic
          const double akk = A[pk][pk], dkk = A[qk][qk], bk = A[pk][qk];
          const double all = A[pl][pl], dll = A[ql][ql], bl = A[pl][ql];
          const double x00 = A[pk][pl], x01 = A[pk][ql], x10 = A[qk][pl], x11 = A[qk][ql];
          double ck, sk, tk, cl, sl, tl;
          jacobi_rotation(akk, dkk, bk, qk < R && !jacobi_discarded(akk, dkk, bk, t2h, t2r), thr,
                          ck, sk, tk);
          jacobi_rotation(all, dll, bl, ql < R && !jacobi_discarded(all, dll, bl, t2h, t2r), thr,
                          cl, sl, tl);
          // rows: J_k^T
          const double y00 = ck * x00 - sk * x10, y01 = ck * x01 - sk * x11;
          const double y10 = sk * x00 + ck * x10, y11 = sk * x01 + ck * x11;
          // columns: J_l
          double z00 = cl * y00 - sl * y01, z01 = sl * y00 + cl * y01;
          double z10 = cl * y10 - sl * y11, z11 = sl * y10 + cl * y11;
          if (k == l && sk != 0.0) {
            // diagonal block: the rotation annihilates the off-diagonal entry
            const double tb = tk * x01;
            z00 = x00 - tb;
            z11 = x11 + tb;
            z01 = 0.0;
            z10 = 0.0;
          }
          // blocks (k, l) and (l, k) are mirror images: write both from one lane
          B[pk][pl] = z00;
          B[pk][ql] = z01;
          B[qk][pl] = z10;
          B[qk][ql] = z11;
          B[pl][pk] = z00;
          B[ql][pk] = z01;
          B[pl][qk] = z10;
          B[ql][qk] = z11;
        }
      } else if (tid >= 64 && tid < 64 + R * half) {
        const int t = tid - 64;
        const int i = t / half, l = t - (t / half) * half;
        int pl, ql;
        rr_pair(rd, l, m, pl, ql);
        const double all = A[pl][pl], dll = A[ql][ql], bl = A[pl][ql];
        const double wp = W[i][pl], wq = W[i][ql];
        double cl, sl, tl;
        jacobi_rotation(all, dll, bl, ql < R && !jacobi_discarded(all, dll, bl, t2h, t2r), thr,
                        cl, sl, tl);
        W[i][pl] = cl * wp - sl * wq;
        W[i][ql] = sl * wp + cl * wq;
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  if (tid == 0) pb.sc->eig_sweeps[n] = sweeps;
  if (tid < kRT) {
    double f = 0.0;
    if (tid < R) {
      const double l = Sb[cur][tid][tid];
      const double sig = sqrt(l > 0.0 ? l : 0.0);
      f = sig > tau ? (sig - tau) / sig : 0.0;
    }
    fac[tid] = f;
    mb.Fac[tid] = f;
  }
  __syncthreads();
  if (tid < 64) {
    const int cnt = __popcll(__ballot(tid < R && fac[tid < kRT ? tid : 0] > 0.0));
    if (tid == 0) pb.sc->rank[n] = cnt;
  }
  {
    const int r = tid / kRT, c = tid % kRT;
    double s = 0.0;
    if (r < R && c < R)
      for (int i = 0; i < R; ++i) s += W[r][i] * fac[i] * W[c][i];
    T1[r][c] = s;
    mb.Wf[tid] = s;
    mb.Wev[tid] = (r < R && c < R) ? W[r][c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // U W_f on the FP64 matrix cores: row block rb (16 rows of U) times W_f
  // (R x 16, zero beyond R), K = 16 in steps of 4; wave w takes blocks w,
  // w + 4, ...  Lane l supplies A[l%16][k] = U[16 rb + l%16][4 s + l/16] and
  // B[k][l%16] = W_f[4 s + l/16][l%16], and ends with rows 4 v + l/16 of
  // column l%16 (the FP64 result layout).
  {
    typedef double d4 __attribute__((ext_vector_type(4)));
    const int lane = tid & 63, wave = tid >> 6;
    const int p = lane & 15, q = lane >> 4;
    const int nrb = (I + 15) / 16;
    double wfb[kRT / 4];
#pragma unroll
    for (int st = 0; st < kRT / 4; ++st) wfb[st] = T1[4 * st + q][p];
    const bool ul = I * R <= kQrLds;
    for (int rb = wave; rb < nrb; rb += 4) {
      const int row = 16 * rb + p;
      const int rc = row < I ? row : I - 1;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < kRT / 4; ++st) {
        const int k = 4 * st + q;
        const int e = rc * R + (k < R ? k : 0);
        const double av = ul ? Ul[e] : mb.U[e];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((row < I && k < R) ? av : 0.0, wfb[st], acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rb + 4 * v + q;
        if (r < I) {
          mb.Uf[(int64_t)r * kRT + p] = (S)acc[v];
          mb.UfT[(int64_t)p * I + r] = (S)acc[v];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Householder QR with the I x R matrix held in registers of one wave: lane l
// owns rows l, l + 64, ..., the column loop is unrolled to RP (R <= RP) so
// every register index is static, and the dot products of one column step
// are reduced together across the wave.
// ---------------------------------------------------------------------------
// Sums K <= 16 values over the 64 lanes of a one-wave block and broadcasts
// the K sums together with K values `row` of lane `src` to every lane.  Lane
// (k, c) = (lane % 16, lane / 16) adds rows 16c..16c+15 of column k from LDS;
// two xor-shuffles combine the four quarters.  The order is fixed.
constexpr int kBatchLds = 64 * 17 + 32;
// kBlock: the wave is the whole block (__syncthreads); otherwise it is one
// wave of a larger block working alone on its own LDS region, where the LDS
// accesses of a wave take effect in program order and only the compiler has
// to be kept from reordering them.
template <bool kBlock>
__device__ __forceinline__ void qr_sync() {
  if constexpr (kBlock) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}
template <int K, bool kBlock = true>
__device__ __forceinline__ void wave_sum_bcast(double (&v)[K], double (&row)[K], int src,
                                               double* lds) {
  constexpr int LD = K + 1;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) lds[lane * LD + k] = v[k];
  if (lane == src) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[64 * 17 + 16 + k] = row[k];
  }
  qr_sync<kBlock>();
  const int k = lane & 15, c = lane >> 4;
  double s = 0;
  if (k < K) {
#pragma unroll
    for (int r = 0; r < 16; ++r) s += lds[(c * 16 + r) * LD + k];
  }
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  if (lane < K) lds[64 * 17 + lane] = s;
  qr_sync<kBlock>();
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    v[kk] = lds[64 * 17 + kk];
    row[kk] = lds[64 * 17 + 16 + kk];
  }
  qr_sync<kBlock>();
}

// One Householder step on column C (compile-time, so every register index is
// static): with d_j = sum_{i > C} a_iC a_ij for j >= C (d_C is the squared norm
// below the diagonal), the reflector v = (1, a_{i>C,C} / (alpha - beta)) gives
// w_j = v^T a_j = a_Cj + d_j / (alpha - beta); one batched reduction per column.
template <int C, int TR, int RP, bool kBlock = true>
__device__ __forceinline__ void qr_factor_col(double (&a)[TR][RP], double (&tau)[RP], int R,
                                              int lane, double* lds) {
  if constexpr (C < RP) {
    if (C < R) {
      constexpr int K = RP - C;
      double d[K], row[K];
#pragma unroll
      for (int jj = 0; jj < K; ++jj) {
        double s = 0;
#pragma unroll
        for (int t = 0; t < TR; ++t)
          if (lane + 64 * t > C) s += a[t][C] * a[t][C + jj];
        d[jj] = s;
        row[jj] = a[0][C + jj];  // row C lives in lane C, slot 0
      }
      wave_sum_bcast<K, kBlock>(d, row, C, lds);
      const double xnorm2 = d[0];
      const double alpha = row[0];
      double tc = 0, beta = alpha, scale = 0;
      if (xnorm2 > 0) {
        // beta = -sgn(alpha) |(alpha, x)|, tau = (beta - alpha) / beta,
        // scale = 1 / (alpha - beta); alpha - beta and beta are nonzero here
        const double n2 = fma(alpha, alpha, xnorm2);
        beta = -copysign(n2 * rsqrt_nr(n2), alpha);
        tc = (beta - alpha) * rcp_nr(beta);
        scale = rcp_nr(alpha - beta);
      }
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const int i = lane + 64 * t;
        const double v = i > C ? a[t][C] * scale : (i == C ? 1.0 : 0.0);
#pragma unroll
        for (int jj = 1; jj < K; ++jj) a[t][C + jj] -= tc * (row[jj] + scale * d[jj]) * v;
        if (i > C) a[t][C] = v;
        if (i == C) a[t][C] = beta;
      }
      tau[C] = tc;
    }
    qr_factor_col<C + 1, TR, RP, kBlock>(a, tau, R, lane, lds);
  }
}

// Backward accumulation of Q = H_0 ... H_{R-1} [I_R; 0], column C down to 0:
// w_j = a_Cj + sum_{i > C} v_i a_ij for j > C, then column C becomes H_C e_C.
template <int C, int TR, int RP, bool kBlock = true>
__device__ __forceinline__ void qr_form_col(double (&a)[TR][RP], const double (&tau)[RP], int R,
                                            int lane, double* lds) {
  if constexpr (C >= 0) {
    if (C < R) {
      const double tc = tau[C];
      constexpr int K = RP - C - 1;
      if constexpr (K > 0) {
        double d[K], row[K];
#pragma unroll
        for (int jj = 0; jj < K; ++jj) {
          double s = 0;
#pragma unroll
          for (int t = 0; t < TR; ++t)
            if (lane + 64 * t > C) s += a[t][C] * a[t][C + 1 + jj];
          d[jj] = s;
          row[jj] = a[0][C + 1 + jj];
        }
        wave_sum_bcast<K, kBlock>(d, row, C, lds);
#pragma unroll
        for (int t = 0; t < TR; ++t) {
          const int i = lane + 64 * t;
          const double v = i > C ? a[t][C] : (i == C ? 1.0 : 0.0);
#pragma unroll
          for (int jj = 0; jj < K; ++jj) a[t][C + 1 + jj] -= tc * (row[jj] + d[jj]) * v;
        }
      }
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const int i = lane + 64 * t;
        a[t][C] = i > C ? -tc * a[t][C] : (i == C ? 1.0 - tc : 0.0);
      }
    }
    qr_form_col<C - 1, TR, RP, kBlock>(a, tau, R, lane, lds);
  }
}

// ---------------------------------------------------------------------------
// Householder QR with the I x R matrix held in registers of one wave: lane l
// owns rows l, l + 64, ...; columns are padded to RP >= R; the dot products
// of one column step are reduced together across the wave.
// ---------------------------------------------------------------------------
template <typename S, int TR, int RP>
__global__ void __launch_bounds__(64) k_qr_reg(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, lane = threadIdx.x;
  // M rows are kRT doubles (16-byte aligned); every lane issues all of its
  // 16-byte loads at once (rows past I clamped, then masked with columns >= R)
  typedef double d2v __attribute__((ext_vector_type(2)));
  double a[TR][RP];
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int i = lane + 64 * t;
    const double* row = mb.M + (int64_t)(i < I ? i : I - 1) * kRT;
#pragma unroll
    for (int c = 0; c < RP; c += 2) {
      const d2v v = *reinterpret_cast<const d2v*>(row + c);
      a[t][c] = (i < I && c < R) ? v[0] : 0.0;
      a[t][c + 1] = (i < I && c + 1 < R) ? v[1] : 0.0;
    }
  }
  __shared__ double lds[kBatchLds];
  double tau[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) tau[c] = 0.0;
  qr_factor_col<0, TR, RP>(a, tau, R, lane, lds);
  qr_form_col<RP - 1, TR, RP>(a, tau, R, lane, lds);
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int i = lane + 64 * t;
    if (i < I) {
#pragma unroll
      for (int c = 0; c < RP; ++c)
        if (c < R) mb.U[(int64_t)i * R + c] = a[t][c];
#pragma unroll
      for (int c = 0; c < kRT; ++c) {
        double v = 0.0;
        if (c < RP)
          v = c < R ? a[t][c < RP ? c : 0] : 0.0;
        mb.Us[(int64_t)i * kRT + c] = (S)v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cholesky QR on the FP64 matrix cores, for I <= 256 and R <= 12: four waves,
// wave w owns rows 64w .. 64w + 63 of the I x R matrix A (first A = M_n).
// One pass:
//   C = A^T A   v_mfma_f64_16x16x4 with both operands the wave's rows (lane
//               (p, q) supplies A[64w + 4s + q][p], four rows per step); the
//               four 16 x 16 partials are summed in LDS in a fixed order;
//   X = R^-1    for C = R^T R, factored in registers by every lane of every
//               wave (the same arithmetic everywhere, so no lane waits for
//               another); each lane then solves for the column of X it
//               supplies to the next product;
//   A <- A X    v_mfma_f64_16x16x4, row block b (16 rows) of the wave times X.
// Two passes are CholeskyQR2 (Yamamoto, Nakatsukasa, Yanagisawa and Fukaya,
// ETNA 44, 2015): with A well conditioned the result is orthonormal to
// rounding; range(A X) = range(A) and R has a positive diagonal, so it is the
// Householder Q up to the signs of its columns.  A pass fails when a pivot
// (the squared norm of column j outside the span of the columns before it) is
// below floor2 times the squared norm of column j: 1e-12 in the first pass
// (column j within 1e-6 of that span), 1/2 in the second (the first result
// far from orthonormal).  Then wave 0 computes the Householder QR of M_n
// instead, which stays orthonormal when M_n is rank deficient, and the other
// waves leave.  Columns j >= R are zero and get r_jj = 1.
// ---------------------------------------------------------------------------
template <int RP>
struct Tri {
  static constexpr int n = RP * (RP + 1) / 2;
  // (j, k), j <= k, in the packed upper triangle stored row by row
  static __device__ __forceinline__ constexpr int at(int j, int k) {
    return j * RP - j * (j - 1) / 2 + (k - j);
  }
};

// c: the upper triangle of C in, of R out (C = R^T R), h[j] = 1 / r_jj.  Row j
// of R is r_jl = (c_jl - sum_{k<j} r_kj r_kl) / r_jj.
template <int RP>
__device__ __forceinline__ bool chol_fact(double (&c)[Tri<RP>::n], double (&h)[RP], int R,
                                          double floor2) {
  bool good = true;
#pragma unroll
  for (int j = 0; j < RP; ++j) {
    const double cjj = c[Tri<RP>::at(j, j)];
    double d = cjj;
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-c[Tri<RP>::at(k, j)], c[Tri<RP>::at(k, j)], d);
    const bool real = j < R;
    good = good && (!real || d > floor2 * cjj);
    const double hj = (real && d > 0.0) ? rsqrt_nr(d) : 1.0;
    h[j] = hj;
#pragma unroll
    for (int l = j + 1; l < RP; ++l) {
      double t = c[Tri<RP>::at(j, l)];
#pragma unroll
      for (int k = 0; k < j; ++k) t = fma(-c[Tri<RP>::at(k, j)], c[Tri<RP>::at(k, l)], t);
      c[Tri<RP>::at(j, l)] = real ? t * hj : 0.0;
    }
    c[Tri<RP>::at(j, j)] = real ? d * hj : 1.0;
  }
  return good;
}

// Column col of X = R^-1 by back substitution, R x = e_col:
// x_i = (delta_i,col - sum_{k>i} r_ik x_k) / r_ii (zero below col; zero
// altogether for col >= RP).
template <int RP>
__device__ __forceinline__ void tri_inv_col(const double (&c)[Tri<RP>::n], const double (&h)[RP],
                                            int col, double (&x)[RP]) {
#pragma unroll
  for (int i = RP - 1; i >= 0; --i) {
    double t = i == col ? 1.0 : 0.0;
#pragma unroll
    for (int k = i + 1; k < RP; ++k) t = fma(-c[Tri<RP>::at(i, k)], x[k], t);
    x[i] = t * h[i];
  }
}

template <typename S, int RP>
__global__ void __launch_bounds__(256) k_qr_chol(Batch<S> bt) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NG = Tri<RP>::n;
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p = lane & 15, q = lane >> 4;
  __shared__ double Cp[4][kRT * kRT];       // per-wave Gram partials
  __shared__ double Cs[kRT * kRT];          // the Gram
  __shared__ double Tw[4][64][kRT + 1];     // a wave's rows, for the change of operand layout
  __shared__ double hl[kBatchLds];          // Householder QR of wave 0
  const double* M = mb.M;
  // every load first (rows clamped into range), then the masks; the wave's
  // 64 x 16 tile also goes to LDS, from where the other operand layout is read
  // (so that it is not held in registers through the factorisation)
  double gA[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int i = 64 * w + 4 * s + q;
    gA[s] = *(const __attribute__((address_space(1))) double*)(M + (int64_t)(i < I ? i : I - 1) * kRT + p);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int i = 64 * w + 4 * s + q;
    gA[s] = (i < I && p < R) ? gA[s] : 0.0;
    Tw[w][4 * s + q][p] = gA[s];
  }
  d4 out[4];
  bool ok = true;
  // not unrolled: one copy of the pass in the instruction stream (these
  // kernels run once per iteration, with a cold instruction cache)
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(gA[s], gA[s], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) Cp[w][(4 * v + q) * kRT + p] = acc[v];
    __syncthreads();
    Cs[tid] = ((Cp[0][tid] + Cp[1][tid]) + Cp[2][tid]) + Cp[3][tid];
    __syncthreads();
    double c[NG];
#pragma unroll
    for (int j = 0; j < RP; ++j)
#pragma unroll
      for (int k = j; k < RP; ++k) c[Tri<RP>::at(j, k)] = Cs[j * kRT + k];
    double h[RP];
    ok = chol_fact<RP>(c, h, R, pass == 0 ? 1e-12 : 0.5);
    ok = __builtin_amdgcn_readfirstlane(ok ? 1 : 0) != 0;
    if (!ok) break;
    // lane (p, q) needs X[4s + q][p]: column p of X, solved in the lane
    double x[RP];
    tri_inv_col<RP>(c, h, p, x);
    double xb[4], aA[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 * s + j < RP) v = q == j ? x[4 * s + j < RP ? 4 * s + j : 0] : v;
      xb[s] = v;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int s = 0; s < 4; ++s) aA[b][s] = Tw[w][16 * b + p][4 * s + q];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      d4 o = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) o = __builtin_amdgcn_mfma_f64_16x16x4f64(aA[b][s], xb[s], o, 0, 0, 0);
      out[b] = o;
    }
    if (pass == 0) {
      // out[b][v] = A[64w + 16b + 4v + q][p]: the Gram layout of the next pass
      // as it stands (s = 4b + v), and the tile for the other layout
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          gA[4 * b + v] = out[b][v];
          Tw[w][16 * b + 4 * v + q][p] = out[b][v];
        }
      qr_sync<false>();
    }
  }
  if (ok) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 64 * w + 16 * b + 4 * v + q;
        if (i < I) {
          if (p < R) mb.U[(int64_t)i * R + p] = out[b][v];
          mb.Us[(int64_t)i * kRT + p] = (S)(p < R ? out[b][v] : 0.0);
        }
      }
    return;
  }
  if (w != 0) return;
  // Householder QR of M_n by wave 0 alone (its own LDS region, no block barrier)
  constexpr int TR = 4;
  typedef double d2v __attribute__((ext_vector_type(2)));
  double a[TR][RP];
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int i = lane + 64 * t;
    const double* row = M + (int64_t)(i < I ? i : I - 1) * kRT;
#pragma unroll
    for (int c = 0; c < RP; c += 2) {
      const d2v v = *reinterpret_cast<const d2v*>(row + c);
      a[t][c] = (i < I && c < R) ? v[0] : 0.0;
      a[t][c + 1] = (i < I && c + 1 < R) ? v[1] : 0.0;
    }
  }
  double tau[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) tau[c] = 0.0;
  qr_factor_col<0, TR, RP, false>(a, tau, R, lane, hl);
  qr_form_col<RP - 1, TR, RP, false>(a, tau, R, lane, hl);
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int i = lane + 64 * t;
    if (i < I) {
#pragma unroll
      for (int c = 0; c < RP; ++c)
        if (c < R) mb.U[(int64_t)i * R + c] = a[t][c];
#pragma unroll
      for (int c = 0; c < kRT; ++c) {
        double v = 0.0;
        if (c < RP) v = c < R ? a[t][c < RP ? c : 0] : 0.0;
        mb.Us[(int64_t)i * kRT + c] = (S)v;
      }
    }
  }
}

template <typename S, int TR>
static bool qr_reg_rp(const Batch<S>& b, int grid, int rmax, hipStream_t s) {
  if (rmax <= 4) {
    hipLaunchKernelGGL((k_qr_reg<S, TR, 4>), dim3(grid), dim3(64), 0, s, b);
  } else if (rmax <= 8) {
    if (TR > 8) return false;
    hipLaunchKernelGGL((k_qr_reg<S, (TR > 8 ? 8 : TR), 8>), dim3(grid), dim3(64), 0, s, b);
  } else if (rmax <= 12) {
    if (TR > 4) return false;
    hipLaunchKernelGGL((k_qr_reg<S, (TR > 4 ? 4 : TR), 12>), dim3(grid), dim3(64), 0, s, b);
  } else {
    if (TR > 4) return false;
    hipLaunchKernelGGL((k_qr_reg<S, (TR > 4 ? 4 : TR), 16>), dim3(grid), dim3(64), 0, s, b);
  }
  return true;
}

// ---------------------------------------------------------------------------
// QR of a tall M_n (R_n <= 16 and I_n R_n above the 8192 doubles the LDS and
// register variants hold), one block of kTallThreads per (problem, mode),
// with A in global memory: M_n's own buffer (rows of kRT doubles, columns
// >= R_n zero), overwritten.  CholeskyQR2 as in k_qr_chol: the Gram on the
// FP64 matrix cores (each wave four rows per MFMA, the wave partials summed in
// LDS in a fixed order), the Cholesky factor and R^-1 by one wave in LDS
// (lane c owns column c), then A <- A R^-1 one row per thread.  A pass fails
// when a pivot is below floor2 times its column's squared norm (1e-12, then
// 1/2, as in k_qr_chol); then the Householder QR of the current A (M_n, or
// the first pass's A R^-1, which still spans range(M_n)) runs on the whole
// block: per column one block-wide batched reduction of the dot products
// (per-wave sums in LDS, summed in wave order) and one update pass, the
// LAPACK dgeqr2 / dorg2r conventions of qr_factor_col / qr_form_col.
// ---------------------------------------------------------------------------
constexpr int kTallThreads = 1024;
constexpr int kTallWaves = kTallThreads / 64;

// Sum part[0..K) over the block (per-wave shuffles, then the waves in order);
// the sums land in out[0..K).  Ends with a barrier.
template <int K>
__device__ __forceinline__ void tall_block_sum(double (&part)[K], double (*red)[kRT + 1],
                                               double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double v = wave_sum(part[j]);
    if (lane == 0) red[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
    for (int v = 0; v < kTallWaves; ++v) t += red[v][threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

template <typename S>
__global__ void __launch_bounds__(kTallThreads) k_qr_tall(Batch<S> bt) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  typedef double d2v __attribute__((ext_vector_type(2)));
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p = lane & 15, q = lane >> 4;
  double* A = mb.M;
  __shared__ double Cp[kTallWaves][kRT * kRT];  // per-wave Gram partials
  __shared__ double C[kRT][kRT + 1];            // the Gram, then R (upper triangle)
  __shared__ double X[kRT][kRT + 1];            // R^-1
  __shared__ double red[kTallWaves][kRT + 1];
  __shared__ double bc[2 * kRT];                // reduced sums, then row c of A
  __shared__ double tauv[kRT];
  __shared__ int bad;
  if (tid == 0) bad = 0;
  for (int pass = 0; pass < 2; ++pass) {
    // C = A^T A: lane (p, q) supplies A[4 st + q][p] to both operands
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    const int nst = (I + 3) / 4;
    constexpr int U = 8;
    for (int s0 = w; s0 < nst; s0 += kTallWaves * U) {
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = 4 * (s0 + kTallWaves * u) + q;
        a[u] = A[(int64_t)(i < I ? i : I - 1) * kRT + p];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = 4 * (s0 + kTallWaves * u) + q;
        const double x = (i < I && p < R) ? a[u] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Cp[w][(4 * v + q) * kRT + p] = acc[v];
    __syncthreads();
    if (tid < kRT * kRT) {
      double t = 0.0;
      for (int v = 0; v < kTallWaves; ++v) t += Cp[v][tid];
      C[tid / kRT][tid % kRT] = t;
    }
    __syncthreads();
    if (w == 0) {
      // right-looking Cholesky C = R^T R on the upper triangle, lane c owns
      // column c; columns >= R get r_cc = 1
      const double floor2 = pass == 0 ? 1e-12 : 0.5;
      const double cdiag = lane < kRT ? C[lane][lane] : 0.0;
      bool good = true;
      for (int j = 0; j < kRT; ++j) {
        // pivot d (row j already reduced by the earlier steps), row j of R,
        // then the rank-one update of the trailing columns, each lane its own
        const double d = C[j][j];
        const bool real = j < R;
        good = good && (!real || d > floor2 * __shfl(cdiag, j, 64));
        const double hj = (real && d > 0.0) ? rsqrt_nr(d) : 1.0;
        const double rjj = (real && d > 0.0) ? d * hj : 1.0;
        const bool mine = lane > j && lane < kRT;
        const double rjl = mine && real ? C[j][lane] * hj : 0.0;
        qr_sync<false>();
        if (mine) C[j][lane] = rjl;
        if (lane == j) C[j][j] = rjj;
        qr_sync<false>();
        if (mine)
          for (int k = j + 1; k <= lane; ++k) C[k][lane] = fma(-C[j][k], rjl, C[k][lane]);
        qr_sync<false>();
      }
      good = __builtin_amdgcn_readfirstlane(good ? 1 : 0) != 0;
      if (!good && lane == 0) bad = 1;
      // X = R^-1, column `lane` by back substitution
      if (lane < kRT) {
        double x[kRT];
#pragma unroll
        for (int i = kRT - 1; i >= 0; --i) {
          double t = i == lane ? 1.0 : 0.0;
#pragma unroll
          for (int k = i + 1; k < kRT; ++k) t = fma(-C[i][k], x[k], t);
          x[i] = i <= lane ? t / C[i][i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kRT; ++i) X[i][lane] = x[i];
      }
    }
    __syncthreads();
    if (bad) break;
    // A <- A X, one row per thread
    for (int i = tid; i < I; i += kTallThreads) {
      double a[kRT];
      const double* row = A + (int64_t)i * kRT;
#pragma unroll
      for (int c = 0; c < kRT; c += 2) {
        const d2v v = *reinterpret_cast<const d2v*>(row + c);
        a[c] = c < R ? v[0] : 0.0;
        a[c + 1] = c + 1 < R ? v[1] : 0.0;
      }
      double o[kRT];
#pragma unroll
      for (int c = 0; c < kRT; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k <= c; ++k) t = fma(a[k], X[k][c], t);
        o[c] = c < R ? t : 0.0;
      }
      if (pass == 0) {
#pragma unroll
        for (int c = 0; c < kRT; ++c) A[(int64_t)i * kRT + c] = o[c];
      } else {
#pragma unroll
        for (int c = 0; c < kRT; ++c) {
          if (c < R) mb.U[(int64_t)i * R + c] = o[c];
          mb.Us[(int64_t)i * kRT + c] = (S)o[c];
        }
      }
    }
    __syncthreads();
  }
  if (!bad) return;
  // Householder QR of A (column-wise, rows of A owned by threads i = tid + kTallThreads k)
  for (int c = 0; c < R; ++c) {
    double part[kRT];
#pragma unroll
    for (int j = 0; j < kRT; ++j) part[j] = 0.0;
    for (int i = c + 1 + tid; i < I; i += kTallThreads) {
      const double* row = A + (int64_t)i * kRT;
      const double ac = row[c];
#pragma unroll
      for (int j = 0; j < kRT; ++j) part[j] = fma(ac, j >= c && j < R ? row[j] : 0.0, part[j]);
    }
    if (tid == 0) {
#pragma unroll
      for (int j = 0; j < kRT; ++j) bc[kRT + j] = A[(int64_t)c * kRT + j];
    }
    tall_block_sum<kRT>(part, red, bc);
    // d_j = bc[j] (j >= c; d_c is the squared norm below the diagonal),
    // row c of A in bc[kRT + j]
    const double xnorm2 = bc[c], alpha = bc[kRT + c];
    double tc = 0.0, beta = alpha, scale = 0.0;
    if (xnorm2 > 0.0) {
      const double n2 = fma(alpha, alpha, xnorm2);
      beta = -copysign(n2 * rsqrt_nr(n2), alpha);
      tc = (beta - alpha) * rcp_nr(beta);
      scale = rcp_nr(alpha - beta);
    }
    for (int i = c + tid; i < I; i += kTallThreads) {
      double* row = A + (int64_t)i * kRT;
      const double v = i > c ? row[c] * scale : 1.0;
      for (int j = c + 1; j < R; ++j) row[j] -= tc * (bc[kRT + j] + scale * bc[j]) * v;
      row[c] = i > c ? v : beta;
    }
    if (tid == 0) tauv[c] = tc;
    __syncthreads();
  }
  // Q = H_0 ... H_{R-1} [I_R; 0], columns R-1 down to 0
  for (int c = R - 1; c >= 0; --c) {
    const double tc = tauv[c];
    double part[kRT];
#pragma unroll
    for (int j = 0; j < kRT; ++j) part[j] = 0.0;
    for (int i = c + 1 + tid; i < I; i += kTallThreads) {
      const double* row = A + (int64_t)i * kRT;
      const double v = row[c];
#pragma unroll
      for (int j = 0; j < kRT; ++j) part[j] = fma(v, j > c && j < R ? row[j] : 0.0, part[j]);
    }
    if (tid == 0) {
#pragma unroll
      for (int j = 0; j < kRT; ++j) bc[kRT + j] = A[(int64_t)c * kRT + j];
    }
    tall_block_sum<kRT>(part, red, bc);
    for (int i = tid; i < I; i += kTallThreads) {
      double* row = A + (int64_t)i * kRT;
      if (i >= c) {
        const double v = i > c ? row[c] : 1.0;
        for (int j = c + 1; j < R; ++j) row[j] -= tc * (bc[kRT + j] + bc[j]) * v;
      }
      row[c] = i > c ? -tc * row[c] : (i == c ? 1.0 - tc : 0.0);
    }
    __syncthreads();
  }
  for (int i = tid; i < I; i += kTallThreads) {
#pragma unroll
    for (int c = 0; c < kRT; ++c) {
      const double v = c < R ? A[(int64_t)i * kRT + c] : 0.0;
      if (c < R) mb.U[(int64_t)i * R + c] = v;
      mb.Us[(int64_t)i * kRT + c] = (S)v;
    }
  }
}

// ---------------------------------------------------------------------------
// Tie-break of eq. (10) that keeps U_n^k on the directions where V_n^k
// vanishes (PASD_FLAG_TIEBREAK_KEEP).  With S = P P^T = W diag(l) W^T from the
// previous eigensolve and f_i its SVT weights, V^k = W diag(f) W^T P^k, so
// G V^T = M W diag(f) W^T with M = G P^T the reduced GEMM-M result; its range
// is spanned by the columns (M W)_i with f_i > 0, and the maximiser of eq. (10)
// nearest U^k completes it on span{(U^k W)_i : f_i = 0}.  Any basis of that
// span serves (the iterates depend on range(U) only), so M is replaced in
// place by the R columns (M W)_i (f_i > 0) and (U^k W)_i (f_i = 0), and the QR
// that follows orthonormalises them.  One block per (problem, mode); a thread
// per row.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_tiebreak(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (!pb.tiebreak_keep || pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, tid = threadIdx.x;
  __shared__ double W[kRT][kRT];
  __shared__ double keep[kRT];  // 1: column i from M W, 0: from U W
  W[tid / kRT][tid % kRT] = mb.Wev[tid];
  if (tid < kRT) keep[tid] = mb.Fac[tid] > 0.0 ? 1.0 : 0.0;
  __syncthreads();
  for (int i = tid; i < I; i += 256) {
    double m[kRT], u[kRT];
#pragma unroll
    for (int c = 0; c < kRT; ++c) {
      m[c] = c < R ? mb.M[(int64_t)i * kRT + c] : 0.0;
      u[c] = c < R ? mb.U[(int64_t)i * R + c] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kRT; ++c) {
      if (c < R) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int r = 0; r < kRT; ++r) {
          a = fma(m[r], W[r][c], a);
          b = fma(u[r], W[r][c], b);
        }
        mb.M[(int64_t)i * kRT + c] = keep[c] != 0.0 ? a : b;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Rank-wide variants (some R_n > kRT; factors stored tile-major, RT = T kRT).
// These carry the same arithmetic as the one-tile kernels with every rank
// index running to R_n <= PASD_MAX_RANK.
// ---------------------------------------------------------------------------
constexpr int kQrLdsW = 16384;  // doubles of LDS for M when R_n > kRT (I_n * R_n <= 16384)
constexpr int kMR = PASD_MAX_RANK;
// The rank-wide QR and eigensolver are latency bound (sequential column steps
// and Jacobi rounds): 512 threads, two waves per SIMD, hide part of it.
constexpr int kWideThreads = 512;
constexpr int kWideWaves = kWideThreads / 64;

// Sum over the threads of a kWideThreads block in a fixed order (red: one
// double of LDS per wave).
__device__ __forceinline__ double block_sum_wide(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kWideWaves; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Applies the reflector of column c (v = (1, scale A[c+1:, c]), tau t) to the
// columns j = c + 1 + wave + kWideWaves u < R that this wave owns: d_j = v^T A[c:, j],
// then A[c:, j] -= t d_j v.  The dot products of all of the wave's columns
// are accumulated and reduced together, without branches (a column index past
// R reads column c and its result is dropped), so a column step costs one
// chain of LDS and shuffle latencies rather than one per column; only the
// stores are conditional.  `wave` must be uniform (readfirstlane).
__device__ __forceinline__ void qrw_reflect(double* A, int I, int R, int c, double t,
                                            double scale, int lane, int wave) {
  constexpr int NU = kMR / kWideWaves;
  int col[NU];
  bool ok[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int j = c + 1 + wave + kWideWaves * u;
    ok[u] = j < R;
    col[u] = (ok[u] ? j : c) * I;
  }
  double d[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) d[u] = 0.0;
  for (int i = c + 1 + lane; i < I; i += 64) {
    const double v = A[c * I + i];
#pragma unroll
    for (int u = 0; u < NU; ++u) d[u] = fma(v, A[col[u] + i], d[u]);
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) d[u] = wave_sum(d[u]);
#pragma unroll
  for (int u = 0; u < NU; ++u) d[u] = ok[u] ? fma(scale, d[u], A[col[u] + c]) : 0.0;
  if (t == 0.0) return;
  for (int i = c + 1 + lane; i < I; i += 64) {
    const double v = A[c * I + i];
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (ok[u]) A[col[u] + i] -= t * d[u] * scale * v;
  }
  if (lane == 0) {
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (ok[u]) A[col[u] + c] -= t * d[u];
  }
}

// CholeskyQR2 for R_n up to kMR (the rank-wide form of k_qr_chol): two passes
// of C = A^T A (FP64 MFMA, tile pairs a <= b), a right-looking Cholesky of C,
// and A <- A R^-1, on A held column-major in LDS.  The factorisation keeps C's
// rows unscaled (after step k, row k holds d_k r_k. / sqrt(d_k), d_k its
// pivot), so a step is one rank-one update of the trailing triangle and one
// barrier; the solve then takes p_j = (a_j - sum_{k<j} p_k c_kj) / d_j along
// each row of A and q_j = p_j sqrt(d_j).  A pivot d_k <= floor2 c_kk (c_kk the
// diagonal before the factorisation; 1e-12 in the first pass, 0.5 in the
// second, as in k_qr_chol) abandons the attempt: A then still spans range(M_n)
// (M_n itself, or the first pass's result) and the Householder QR takes over.
// Returns whether both passes succeeded (block-uniform).
constexpr int kCholW = kQrLdsW - kMR * (kMR + 1);  // I_n R_n limit: A and C share the LDS
__device__ __forceinline__ bool qrw_cholqr2(double* A, double (*C)[kMR + 1], double* c0,
                                            double* piv, int I, int R, int T, int tid, int lane,
                                            int wave) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int kSlots = (kMR * (kMR + 1) / 2 + kWideThreads - 1) / kWideThreads;
  // upper-triangle entries (i, j), i <= j < R, owned by this thread
  int si[kSlots], sj[kSlots];
  const int ntri = R * (R + 1) / 2;
#pragma unroll
  for (int u = 0; u < kSlots; ++u) {
    int e = tid + kWideThreads * u, i = 0;
    if (e >= ntri) e = ntri - 1;
    while (e >= R - i) {
      e -= R - i;
      ++i;
    }
    si[u] = i;
    sj[u] = i + e;
  }
  for (int pass = 0; pass < 2; ++pass) {
    const double floor2 = pass == 0 ? 1e-12 : 0.5;
    // C = A^T A on the FP64 MFMA: lane (p, q) = (lane % 16, lane / 16) supplies
    // A[k0 + q][16 a + p] for the A operand and A[k0 + q][16 b + p] for B.
    const int p = lane & 15, q = lane >> 4;
    const int np = T * (T + 1) / 2;
    for (int pr = wave; pr < np; pr += kWideWaves) {
      int a = 0, b = pr;
      while (b >= T - a) {
        b -= T - a;
        ++a;
      }
      b += a;
      const int ca = 16 * a + p, cb = 16 * b + p;
      const double* xa = A + (int64_t)min(ca, R - 1) * I;
      const double* xb = A + (int64_t)min(cb, R - 1) * I;
      const bool oka = ca < R, okb = cb < R;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < I; k0 += 16) {
        double va[4], vb[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int row = min(k0 + 4 * s4 + q, I - 1);
          va[s4] = xa[row];
          vb[s4] = xb[row];
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const bool rok = k0 + 4 * s4 + q < I;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((rok && oka) ? va[s4] : 0.0,
                                                     (rok && okb) ? vb[s4] : 0.0, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) C[16 * a + 4 * v + q][16 * b + p] = acc[v];
    }
    __syncthreads();
    if (tid < R) c0[tid] = C[tid][tid];
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < R; ++k) {
      const double d = C[k][k];
      if (!(d > floor2 * c0[k])) {
        ok = false;
        break;
      }
      const double rd = 1.0 / d;
      double ck[kSlots], cj[kSlots];
#pragma unroll
      for (int u = 0; u < kSlots; ++u) {
        ck[u] = C[k][si[u]];
        cj[u] = C[k][sj[u]];
      }
#pragma unroll
      for (int u = 0; u < kSlots; ++u)
        if (tid + kWideThreads * u < ntri && si[u] > k) C[si[u]][sj[u]] -= ck[u] * cj[u] * rd;
      __syncthreads();
    }
    if (!ok) return false;
    if (tid < R) piv[tid] = C[tid][tid];
    __syncthreads();
    for (int i = tid; i < I; i += kWideThreads) {
      for (int j = 0; j < R; ++j) {
        double a0 = A[j * I + i], a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int k = 0;
        for (; k + 4 <= j; k += 4) {
          a0 = fma(-A[k * I + i], C[k][j], a0);
          a1 = fma(-A[(k + 1) * I + i], C[k + 1][j], a1);
          a2 = fma(-A[(k + 2) * I + i], C[k + 2][j], a2);
          a3 = fma(-A[(k + 3) * I + i], C[k + 3][j], a3);
        }
        for (; k < j; ++k) a0 = fma(-A[k * I + i], C[k][j], a0);
        A[j * I + i] = ((a0 + a1) + (a2 + a3)) / piv[j];
      }
      for (int j = 0; j < R; ++j) A[j * I + i] *= sqrt(piv[j]);
    }
    __syncthreads();
  }
  return true;
}

// QR of M_n for R_n > kRT (column-major in LDS): CholeskyQR2 (qrw_cholqr2)
// where I_n R_n <= kCholW and both passes keep their pivots, else Householder
// QR by the whole block, the same reflectors as k_qr (LAPACK dgeqr2 / dorg2r
// conventions): wave w applies the
// reflector of a column step to columns c + 1 + w, c + 1 + w + kWideWaves, ...
// (qrw_reflect), each a wave-wide dot product followed by its update, so the
// waves need no barrier between the two.  A factorisation step has one
// barrier: the reflector's scale is applied on the fly (the stored column is
// scaled, and its diagonal and tau written, during the next step, which does
// not read it), and wave 0, which owns column c + 1, forms that column's norm
// right after updating it (double-buffered, as the other waves may still be
// reading the previous one).
template <typename S>
__global__ void __launch_bounds__(kWideThreads) k_qr_w(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, T = g.T, tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ double A[kQrLdsW];  // column-major A[c * I + i]
  __shared__ double tau[kMR];
  __shared__ double red[kWideWaves];
  __shared__ double nrm[2];  // squared norm below the diagonal of the next column
  __shared__ double c0[kMR], piv[kMR];
  for (int e = tid; e < I * R; e += kWideThreads) {
    const int c = e / I, i = e - c * I;
    A[e] = mb.M[((int64_t)(c / kRT) * I + i) * kRT + c % kRT];
  }
  __syncthreads();
  bool done = false;
  if (I * R <= kCholW)
    done = qrw_cholqr2(A, reinterpret_cast<double (*)[kMR + 1]>(A + kCholW), c0, piv, I, R, T, tid,
                       lane, wave);
  if (!done) {
    {
      double part = 0;
      for (int i = 1 + tid; i < I; i += kWideThreads) {
        const double x = A[i];
        part += x * x;
      }
      part = block_sum_wide(part, red);
      if (tid == 0) nrm[0] = part;
      __syncthreads();
    }
    double pscale = 1.0, pbeta = 0.0, pt = 0.0;  // step c - 1, applied during step c
    for (int c = 0; c < R; ++c) {
      if (c > 0) {
        if (pscale != 1.0)
          for (int i = c + tid; i < I; i += kWideThreads) A[(c - 1) * I + i] *= pscale;
        if (tid == 0) {
          A[(c - 1) * I + c - 1] = pbeta;
          tau[c - 1] = pt;
        }
      }
      const double xnorm2 = nrm[c & 1];
      const double alpha = A[c * I + c];
      double t = 0, beta = alpha, scale = 0;
      if (xnorm2 > 0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      qrw_reflect(A, I, R, c, t, scale, lane, wave);
      if (wave == 0 && c + 1 < R) {
        double part = 0;
        for (int i = c + 2 + lane; i < I; i += 64) {
          const double x = A[(c + 1) * I + i];
          part += x * x;
        }
        part = wave_sum(part);
        if (lane == 0) nrm[(c + 1) & 1] = part;
      }
      pscale = xnorm2 > 0 ? scale : 1.0;
      pbeta = beta;
      pt = t;
      __syncthreads();
    }
    if (pscale != 1.0)
      for (int i = R + tid; i < I; i += kWideThreads) A[(R - 1) * I + i] *= pscale;
    if (tid == 0) {
      A[(R - 1) * I + R - 1] = pbeta;
      tau[R - 1] = pt;
    }
    __syncthreads();
    for (int c = R - 1; c >= 0; --c) {
      const double t = tau[c];
      qrw_reflect(A, I, R, c, t, 1.0, lane, wave);
      __syncthreads();
      for (int i = c + 1 + tid; i < I; i += kWideThreads) A[c * I + i] = -t * A[c * I + i];
      if (tid == 0) A[c * I + c] = 1.0 - t;
      for (int i = tid; i < c; i += kWideThreads) A[c * I + i] = 0.0;
      __syncthreads();
    }
  }  // Householder
  for (int e = tid; e < I * T * kRT; e += kWideThreads) {
    const int t = e / (I * kRT), rem = e - t * I * kRT;
    const int i = rem / kRT, c = t * kRT + rem % kRT;
    const double v = c < R ? A[c * I + i] : 0.0;
    if (c < R) mb.U[(int64_t)i * R + c] = v;
    mb.Us[e] = (S)v;
  }
}

// The keep tie-break transform of M_n (see k_tiebreak) for R_n up to kMR: rows
// of M_n and U_n are staged in LDS 64 at a time, thread (row, column) forms
// both candidates and keeps one.
template <typename S>
__global__ void __launch_bounds__(256) k_tiebreak_w(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (!pb.tiebreak_keep || pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int I = g.I, R = g.R, RT = g.T * kRT, tid = threadIdx.x;
  __shared__ double W[kMR][kMR + 1];
  __shared__ double keep[kMR];
  __shared__ double Ml[64][kMR];
  __shared__ double Ul[64][kMR];
  for (int e = tid; e < RT * RT; e += 256) W[e / RT][e % RT] = mb.Wev[e];
  for (int e = tid; e < RT; e += 256) keep[e] = mb.Fac[e] > 0.0 ? 1.0 : 0.0;
  const int c = tid & 63;
  for (int i0 = 0; i0 < I; i0 += 64) {
    const int ni = min(64, I - i0);
    __syncthreads();
    for (int e = tid; e < ni * R; e += 256) {
      const int il = e / R, r = e - il * R, i = i0 + il;
      Ml[il][r] = mb.M[((int64_t)(r / kRT) * I + i) * kRT + r % kRT];
      Ul[il][r] = mb.U[(int64_t)i * R + r];
    }
    __syncthreads();
    if (c < R) {
      for (int il = tid >> 6; il < ni; il += 4) {
        double a = 0.0, b = 0.0;
        for (int r = 0; r < R; ++r) {
          a = fma(Ml[il][r], W[r][c], a);
          b = fma(Ul[il][r], W[r][c], b);
        }
        mb.M[((int64_t)(c / kRT) * I + i0 + il) * kRT + c % kRT] = keep[c] != 0.0 ? a : b;
      }
    }
  }
}

// The SVT factor for R_n up to kMR (steps of k_eig): the Gram from its
// partials, the warm start S' = W0^T S W0, round-robin Jacobi sweeps until no
// pair needs a rotation, then W_f = W diag(f) W^T and U W_f.  A round computes
// the R'/2 rotations once (one thread per pair, into LDS), then every thread
// applies them to its 2 x 2 blocks (k, l), k <= l, of the matrix (read from
// one buffer, written to the other; only the upper triangle is kept, which
// halves the LDS writes of a round) and to its entries of the eigenvectors.
// Each thread has fixed slots (block tid + kWideThreads u, eigenvector entry
// tid + kWideThreads u)
// whose indices are clamped into range, so that all reads of a phase are
// issued together; only the writes of valid slots happen.
constexpr int kEigBlk = (kMR / 2) * (kMR / 2 + 1) / 2;  // blocks (k, l), k <= l
constexpr int kEigBU = (kEigBlk + kWideThreads - 1) / kWideThreads;
constexpr int kEigWU = (kMR * (kMR / 2) + kWideThreads - 1) / kWideThreads;
template <typename S>
__global__ void __launch_bounds__(kWideThreads) k_eig_w(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int n = blockIdx.x - bt.start[req];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int R = g.R, I = g.I, RT = g.T * kRT, tid = threadIdx.x;
  const bool warm = pb.sc->k > 0;
  __shared__ double Sb[2][kMR][kMR + 1];
  __shared__ double W[kMR][kMR + 1];
  __shared__ double T1[kMR][kMR + 1];
  __shared__ double rot[kMR / 2][3];
  __shared__ double fac[kMR];
  __shared__ int blk_kl[kEigBlk];  // (k << 8) | l of block slot e
  __shared__ unsigned long long rmask[2];  // rounds of the coming sweep with a pair to rotate
  const int nb = mb.sblocks;
  for (int e = tid; e < RT * RT; e += kWideThreads) {
    const int r = e / RT, c = e - r * RT;
    const bool in = r < R && c < R;
    double sm = 0.0;
#pragma unroll 8
    for (int b = 0; b < nb; ++b) sm += mb.Spart[(int64_t)b * RT * RT + e];
    Sb[0][r][c] = in ? sm : 0.0;
    W[r][c] = (warm && in) ? mb.Wev[e] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int e = tid; e < RT * RT; e += kWideThreads) {  // T1 = S W0, S from its upper triangle
    const int r = e / RT, c = e - r * RT;
    double t = 0;
    for (int k = 0; k < R; ++k) t += (r <= k ? Sb[0][r][k] : Sb[0][k][r]) * W[k][c];
    T1[r][c] = t;
  }
  __syncthreads();
  for (int e = tid; e < RT * RT; e += kWideThreads) {  // S' = W0^T T1, symmetric by construction
    const int r = e / RT, c = e - r * RT;
    const int rr = r <= c ? r : c, cc = r <= c ? c : r;
    double v = 0;
    for (int k = 0; k < R; ++k) v += W[k][rr] * T1[k][cc];
    Sb[1][r][c] = (r < R && c < R) ? v : 0.0;
  }
  __syncthreads();
  const double thr = sizeof(S) == 4 ? 5.9604644775390625e-08 : 4.0e-16;
  const double tau = pb.lam[n] / pb.sc->mu;
  const double t2h = 0.5 * tau * tau, t2r = t2h / R;
  const int Rp = R + (R & 1);
  const int half = Rp / 2;
  const int m = Rp - 1;
  const int nblk = half * (half + 1) / 2;
  const int nwe = R * half;
  // i = e / half for e < kMR * kMR / 2 by multiply and shift: with
  // mh = ceil(2^16 / half) the error of e mh / 2^16 is below 2048 / 2^16 = 1/32,
  // and the fractional part of e / half is at most 1 - 1/half <= 1 - 1/32
  const int mh = half > 0 ? (65536 + half - 1) / half : 0;
  for (int e = tid; e < nblk; e += kWideThreads) {
    int k = 0, rem = e;
    while (rem >= half - k) {
      rem -= half - k;
      ++k;
    }
    blk_kl[e] = (k << 8) | (k + rem);
  }
  __syncthreads();
  // this thread's slots, the same in every round: blocks (k, l) and
  // eigenvector entries (row i, pair l)
  int bk[kEigBU], bl[kEigBU], wi[kEigWU], wl[kEigWU];
#pragma unroll
  for (int u = 0; u < kEigBU; ++u) {
    const int kl = blk_kl[min(tid + kWideThreads * u, nblk - 1)];
    bk[u] = kl >> 8;
    bl[u] = kl & 255;
  }
#pragma unroll
  for (int u = 0; u < kEigWU; ++u) {
    const int e = min(tid + kWideThreads * u, nwe - 1);
    wi[u] = (e * mh) >> 16;
    wl[u] = e - wi[u] * half;
  }
  int sweeps = 0;
  int cur = 1;
  if (tid < 2) rmask[tid] = 0ull;
  __syncthreads();
  for (int sweep = 0; sweep < 40 && R > 1; ++sweep) {
    int need = 0;
    unsigned long long bits = 0ull;
    for (int e = tid; e < R * R; e += kWideThreads) {
      const int p = e / R, q = e - p * R;
      if (p < q &&
          jacobi_needed(Sb[cur], p, q, thr) &&
          !jacobi_discarded(Sb[cur][p][p], Sb[cur][q][q], Sb[cur][p][q], t2h, t2r)) {
        need = 1;
        bits |= 1ull << rr_round(p, q, m);
      }
    }
    if (bits) atomicOr(&rmask[sweep & 1], bits);
    if (!__syncthreads_or(need)) break;
    sweeps = sweep + 1;
    // rounds whose pairs all passed the check are skipped (see k_eig)
    const unsigned long long mask = rmask[sweep & 1];
    if (tid == 0) rmask[(sweep + 1) & 1] = 0ull;
    for (int rd = 0; rd < m; ++rd) {
      if (!((mask >> rd) & 1ull)) continue;
      const double (*A)[kMR + 1] = Sb[cur];
      double (*B)[kMR + 1] = Sb[cur ^ 1];
      if (tid < half) {
        int p, q;
        rr_pair(rd, tid, m, p, q);
        double c, sn, t;
        const double app = A[p][p], aqq = A[q][q], apq = A[p][q];
        jacobi_rotation(app, aqq, apq, q < R && !jacobi_discarded(app, aqq, apq, t2h, t2r), thr, c,
                        sn, t);
        rot[tid][0] = c;
        rot[tid][1] = sn;
        rot[tid][2] = t;
      }
      __syncthreads();
      {
        int pk[kEigBU], qk[kEigBU], pl[kEigBU], ql[kEigBU];
        bool diag[kEigBU];
        double ck[kEigBU], sk[kEigBU], tk[kEigBU], cl[kEigBU], sl[kEigBU], x[kEigBU][4];
#pragma unroll
        for (int u = 0; u < kEigBU; ++u) {
          const int k = bk[u], l = bl[u];
          diag[u] = k == l;
          rr_pair(rd, k, m, pk[u], qk[u]);
          rr_pair(rd, l, m, pl[u], ql[u]);
          ck[u] = rot[k][0];
          sk[u] = rot[k][1];
          tk[u] = rot[k][2];
          cl[u] = rot[l][0];
          sl[u] = rot[l][1];
          // the rotated matrix is kept in its upper triangle only
          x[u][0] = A[min(pk[u], pl[u])][max(pk[u], pl[u])];
          x[u][1] = A[min(pk[u], ql[u])][max(pk[u], ql[u])];
          x[u][2] = A[min(qk[u], pl[u])][max(qk[u], pl[u])];
          x[u][3] = A[min(qk[u], ql[u])][max(qk[u], ql[u])];
        }
        int pw[kEigWU], qw[kEigWU], iw[kEigWU];
        double cw[kEigWU], sw[kEigWU], wp[kEigWU], wq[kEigWU];
#pragma unroll
        for (int u = 0; u < kEigWU; ++u) {
          const int i = wi[u], l = wl[u];
          iw[u] = i;
          rr_pair(rd, l, m, pw[u], qw[u]);
          cw[u] = rot[l][0];
          sw[u] = rot[l][1];
          wp[u] = W[i][pw[u]];
          wq[u] = W[i][qw[u]];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kEigBU; ++u) {
          if (tid + kWideThreads * u >= nblk) continue;
          const double x00 = x[u][0], x01 = x[u][1], x10 = x[u][2], x11 = x[u][3];
          const double y00 = ck[u] * x00 - sk[u] * x10, y01 = ck[u] * x01 - sk[u] * x11;
          const double y10 = sk[u] * x00 + ck[u] * x10, y11 = sk[u] * x01 + ck[u] * x11;
          double z00 = cl[u] * y00 - sl[u] * y01, z01 = sl[u] * y00 + cl[u] * y01;
          double z10 = cl[u] * y10 - sl[u] * y11, z11 = sl[u] * y10 + cl[u] * y11;
          if (diag[u] && sk[u] != 0.0) {
            const double tb = tk[u] * x01;
            z00 = x00 - tb;
            z11 = x11 + tb;
            z01 = 0.0;
            z10 = 0.0;
          }
          B[min(pk[u], pl[u])][max(pk[u], pl[u])] = z00;
          B[min(pk[u], ql[u])][max(pk[u], ql[u])] = z01;
          B[min(qk[u], pl[u])][max(qk[u], pl[u])] = z10;
          B[min(qk[u], ql[u])][max(qk[u], ql[u])] = z11;
        }
#pragma unroll
        for (int u = 0; u < kEigWU; ++u) {
          if (tid + kWideThreads * u >= nwe) continue;
          W[iw[u]][pw[u]] = cw[u] * wp[u] - sw[u] * wq[u];
          W[iw[u]][qw[u]] = sw[u] * wp[u] + cw[u] * wq[u];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  if (tid == 0) pb.sc->eig_sweeps[n] = sweeps;
  if (tid < RT) {
    double f = 0.0;
    if (tid < R) {
      const double l = Sb[cur][tid][tid];
      const double sig = sqrt(l > 0.0 ? l : 0.0);
      f = sig > tau ? (sig - tau) / sig : 0.0;
    }
    fac[tid] = f;
    mb.Fac[tid] = f;
  }
  __syncthreads();
  if (tid < 64) {
    const int cnt = __popcll(__ballot(tid < R && fac[tid] > 0.0));
    if (tid == 0) pb.sc->rank[n] = cnt;
  }
  for (int e = tid; e < RT * RT; e += kWideThreads) {
    const int r = e / RT, c = e - r * RT;
    double sm = 0.0;
    if (r < R && c < R)
      for (int i = 0; i < R; ++i) sm += W[r][i] * fac[i] * W[c][i];
    T1[r][c] = sm;
    mb.Wf[e] = sm;
    mb.Wev[e] = (r < R && c < R) ? W[r][c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // U W_f: lane c is a column of the result, wave w takes rows w, w + kWideWaves, ...
  const int c = tid & 63;
  if (c < RT) {
    for (int i = tid >> 6; i < I; i += kWideWaves) {
      const double* urow = mb.U + (int64_t)i * R;
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < R; ++k) acc = fma(urow[k], T1[k][c], acc);
      mb.Uf[((int64_t)(c / kRT) * I + i) * kRT + c % kRT] = (S)acc;
      mb.UfT[(int64_t)c * I + i] = (S)acc;
    }
  }
}

// One wave per (problem, mode); the register variant is sized for the largest
// I_n and R_n of the set, the LDS variant takes what does not fit.  With the
// keep tie-break on any problem of the set, its transform of M_n runs first.
// Problems with a tall mode (I_n R_n > kQrLds) take k_qr_tall for every mode.
template <typename S>
static bool has_tall_mode(const Problem<S>& p) {
  for (int n = 0; n < p.N; ++n)
    if (p.g[n].I * p.g[n].R > kQrLds) return true;
  return false;
}

template <typename S>
static void launch_qr_narrow(const LaunchSet<S>& all, hipStream_t s) {
  LaunchSet<S> ls, tall;
  ls.count = tall.count = 0;
  for (int r = 0; r < all.count; ++r) {
    LaunchSet<S>& d = has_tall_mode(*all.host[r]) ? tall : ls;
    d.host[d.count] = all.host[r];
    d.dev[d.count] = all.dev[r];
    ++d.count;
  }
  Batch<S> b;
  if (tall.count) {
    const int grid = make_batch(tall, b, [](const Problem<S>& p) { return p.N; });
    bool keep = false;
    for (int r = 0; r < tall.count; ++r) keep = keep || tall.host[r]->tiebreak_keep;
    if (keep) hipLaunchKernelGGL(k_tiebreak<S>, dim3(grid), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_qr_tall<S>, dim3(grid), dim3(kTallThreads), 0, s, b);
  }
  if (!ls.count) return;
  const int grid = make_batch(ls, b, [](const Problem<S>& p) { return p.N; });
  bool keep = false;
  for (int r = 0; r < ls.count; ++r) keep = keep || ls.host[r]->tiebreak_keep;
  if (keep) hipLaunchKernelGGL(k_tiebreak<S>, dim3(grid), dim3(256), 0, s, b);
  int imax = 1, rmax = 1;
  for (int r = 0; r < ls.count; ++r)
    for (int n = 0; n < ls.host[r]->N; ++n) {
      imax = ls.host[r]->g[n].I > imax ? ls.host[r]->g[n].I : imax;
      rmax = ls.host[r]->g[n].R > rmax ? ls.host[r]->g[n].R : rmax;
    }
  bool done = false;
  if (imax <= 256 && rmax <= 12) {
    // the factorisation is unrolled to R rounded up to even
    switch ((rmax + 1) / 2) {
      case 1:
      case 2: hipLaunchKernelGGL((k_qr_chol<S, 4>), dim3(grid), dim3(256), 0, s, b); return;
      case 3: hipLaunchKernelGGL((k_qr_chol<S, 6>), dim3(grid), dim3(256), 0, s, b); return;
      case 4: hipLaunchKernelGGL((k_qr_chol<S, 8>), dim3(grid), dim3(256), 0, s, b); return;
      case 5: hipLaunchKernelGGL((k_qr_chol<S, 10>), dim3(grid), dim3(256), 0, s, b); return;
      default: hipLaunchKernelGGL((k_qr_chol<S, 12>), dim3(grid), dim3(256), 0, s, b); return;
    }
  }
  if (imax <= 64)
    done = qr_reg_rp<S, 1>(b, grid, rmax, s);
  else if (imax <= 128)
    done = qr_reg_rp<S, 2>(b, grid, rmax, s);
  else if (imax <= 256)
    done = qr_reg_rp<S, 4>(b, grid, rmax, s);
  else if (imax <= 512)
    done = qr_reg_rp<S, 8>(b, grid, rmax, s);
  else if (imax <= 1024)
    done = qr_reg_rp<S, 16>(b, grid, rmax, s);
  if (!done) hipLaunchKernelGGL(k_qr<S>, dim3(grid), dim3(64), 0, s, b);
}

template <typename S>
void launch_qr(const LaunchSet<S>& ls, hipStream_t s) {
  LaunchSet<S> nar, wid;
  split_wide(ls, nar, wid);
  if (nar.count) launch_qr_narrow(nar, s);
  if (wid.count) {
    Batch<S> b;
    const int grid = make_batch(wid, b, [](const Problem<S>& p) { return p.N; });
    bool keep = false;
    for (int r = 0; r < wid.count; ++r) keep = keep || wid.host[r]->tiebreak_keep;
    if (keep) hipLaunchKernelGGL(k_tiebreak_w<S>, dim3(grid), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_qr_w<S>, dim3(grid), dim3(kWideThreads), 0, s, b);
  }
}

template <typename S>
void launch_eig(const LaunchSet<S>& ls, hipStream_t s) {
  LaunchSet<S> nar, wid;
  split_wide(ls, nar, wid);
  Batch<S> b;
  if (nar.count) {
    const int grid = make_batch(nar, b, [](const Problem<S>& p) { return p.N; });
    hipLaunchKernelGGL(k_eig<S>, dim3(grid), dim3(256), 0, s, b);
  }
  if (wid.count) {
    const int grid = make_batch(wid, b, [](const Problem<S>& p) { return p.N; });
    hipLaunchKernelGGL(k_eig_w<S>, dim3(grid), dim3(kWideThreads), 0, s, b);
  }
}

template void launch_qr<float>(const LaunchSet<float>&, hipStream_t);
template void launch_qr<double>(const LaunchSet<double>&, hipStream_t);
template void launch_eig<float>(const LaunchSet<float>&, hipStream_t);
template void launch_eig<double>(const LaunchSet<double>&, hipStream_t);

}  // namespace pasd
