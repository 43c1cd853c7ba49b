// Small per-mode FP64 kernels of the PASD iteration, one 64-lane wave per mode.
//
//   k_qr  : U_n = Q of the Householder QR of M_n = G_n P_n^T.  range(U_n) is the
//           range of the Procrustes solution of eqs. (9)-(10); the iterates
//           depend on range(U_n) only, so any orthonormal basis of it will do.
//           Householder QR stays orthonormal when M_n is rank deficient.
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
__global__ void __launch_bounds__(64) k_qr(Problem<S> pb) {
  if (pb.sc->done || pb.sc->k == 0) return;
  const int n = blockIdx.x;
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
// Parallel cyclic Jacobi on the R x R Gram (R <= 16), round-robin pairing:
// every round rotates R'/2 disjoint pairs (R' = R rounded up to even, a dummy
// index for odd R).  One lane per 2x2 block applies J_k^T S J_l.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(64) k_eig(Problem<S> pb) {
  if (pb.sc->done) return;
  const int n = blockIdx.x;
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int R = g.R, lane = threadIdx.x;
  __shared__ double Sm[kRT][kRT + 1];
  __shared__ double W[kRT][kRT + 1];
  __shared__ double cs[kRT / 2][2];
  __shared__ int pq[kRT / 2][2];
  __shared__ double fac[kRT];
  __shared__ double Wf[kRT][kRT + 1];
  for (int e = lane; e < kRT * kRT; e += 64) {
    const int r = e / kRT, c = e - r * kRT;
    double s = 0;
    if (r < R && c < R)
      for (int b = 0; b < mb.sblocks; ++b) s += mb.Spart[(int64_t)b * kRT * kRT + e];
    Sm[r][c] = s;
    W[r][c] = (r == c) ? 1.0 : 0.0;
  }
  // symmetrise (the two triangles are summed in the same order, but be exact)
  __syncthreads();
  for (int e = lane; e < kRT * kRT; e += 64) {
    const int r = e / kRT, c = e - r * kRT;
    if (r > c) Sm[r][c] = Sm[c][r];
  }
  __syncthreads();
  const int Rp = R + (R & 1);
  const int half = Rp / 2;
  const int m = Rp - 1;
  for (int sweep = 0; sweep < 40 && Rp > 1; ++sweep) {
    int rotated = 0;
    for (int rd = 0; rd < m; ++rd) {
      if (lane < half) {
        int p, q;
        if (lane == 0) {
          p = m;
          q = rd;
        } else {
          p = (rd + lane) % m;
          q = (rd - lane + m) % m;
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0;
        if (q < R) {
          const double a = Sm[p][p], d = Sm[q][q], b = Sm[p][q];
          const double ab = fabs(b);
          if (ab > 1e-300 && ab > 4.0e-16 * sqrt(fabs(a)) * sqrt(fabs(d))) {
            const double th = (d - a) / (2.0 * b);
            const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            rotated = 1;
          }
        }
        cs[lane][0] = c;
        cs[lane][1] = s;
        pq[lane][0] = p;
        pq[lane][1] = q;
      }
      rotated = __syncthreads_or(rotated);
      if (lane < half * half && lane / half <= lane % half) {
        const int k = lane / half, l = lane - k * half;
        const int pk = pq[k][0], qk = pq[k][1], pl = pq[l][0], ql = pq[l][1];
        const double ck = cs[k][0], sk = cs[k][1], cl = cs[l][0], sl = cs[l][1];
        const double x00 = Sm[pk][pl], x01 = Sm[pk][ql], x10 = Sm[qk][pl], x11 = Sm[qk][ql];
        // rows: J_k^T
        const double y00 = ck * x00 - sk * x10, y01 = ck * x01 - sk * x11;
        const double y10 = sk * x00 + ck * x10, y11 = sk * x01 + ck * x11;
        // columns: J_l
        double z00 = cl * y00 - sl * y01, z01 = sl * y00 + cl * y01;
        double z10 = cl * y10 - sl * y11, z11 = sl * y10 + cl * y11;
        if (k == l && sk != 0.0) {
          // diagonal block: the rotation annihilates the off-diagonal entry
          const double b = x01;
          const double t = sk / ck;
          z00 = x00 - t * b;
          z11 = x11 + t * b;
          z01 = 0.0;
          z10 = 0.0;
        }
        // blocks (k, l) and (l, k) are mirror images: write both from one lane
        Sm[pk][pl] = z00;
        Sm[pk][ql] = z01;
        Sm[qk][pl] = z10;
        Sm[qk][ql] = z11;
        Sm[pl][pk] = z00;
        Sm[ql][pk] = z01;
        Sm[pl][qk] = z10;
        Sm[ql][qk] = z11;
      }
      for (int e = lane; e < kRT * half; e += 64) {
        const int i = e / half, l = e - i * half;
        const int pl = pq[l][0], ql = pq[l][1];
        const double cl = cs[l][0], sl = cs[l][1];
        const double wp = W[i][pl], wq = W[i][ql];
        W[i][pl] = cl * wp - sl * wq;
        W[i][ql] = sl * wp + cl * wq;
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  const double tau = pb.lam[n] / pb.sc->mu;
  if (lane < kRT) {
    double f = 0.0;
    if (lane < R) {
      const double l = Sm[lane][lane];
      const double sig = sqrt(l > 0.0 ? l : 0.0);
      f = sig > tau ? (sig - tau) / sig : 0.0;
    }
    fac[lane] = f;
  }
  __syncthreads();
  {
    int cnt = (lane < R && fac[lane] > 0.0) ? 1 : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) pb.sc->rank[n] = cnt;
  }
  for (int e = lane; e < kRT * kRT; e += 64) {
    const int r = e / kRT, c = e - r * kRT;
    double s = 0.0;
    if (r < R && c < R)
      for (int i = 0; i < R; ++i) s += W[r][i] * fac[i] * W[c][i];
    Wf[r][c] = s;
    mb.Wf[e] = s;
  }
  __syncthreads();
  const int I = g.I;
  for (int e = lane; e < I * kRT; e += 64) {
    const int i = e / kRT, c = e - i * kRT;
    double s = 0.0;
    if (c < R)
      for (int r = 0; r < R; ++r) s += mb.U[(int64_t)i * R + r] * Wf[r][c];
    mb.Uf[e] = (S)s;
    mb.UfT[(int64_t)c * I + i] = (S)s;
  }
}

template <typename S>
void launch_qr(const Problem<S>& p, hipStream_t s) {
  hipLaunchKernelGGL(k_qr<S>, dim3(p.N), dim3(64), 0, s, p);
}

template <typename S>
void launch_eig(const Problem<S>& p, hipStream_t s) {
  hipLaunchKernelGGL(k_eig<S>, dim3(p.N), dim3(64), 0, s, p);
}

template void launch_qr<float>(const Problem<float>&, hipStream_t);
template void launch_qr<double>(const Problem<double>&, hipStream_t);
template void launch_eig<float>(const Problem<float>&, hipStream_t);
template void launch_eig<double>(const Problem<double>&, hipStream_t);

}  // namespace pasd
