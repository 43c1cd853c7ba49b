// Elementwise passes of the PASD iteration.
//
// k_fused makes one coalesced pass over the tensor per iteration.  For every
// element x and mode n it forms Z_n(x) = (U_n W_n)[i_n(x), :] . P_n[:, j_n(x)]
// (Algorithm 1, line 5, with V_n = W_n P_n), then
//   E(x)  = prox_{1/(mu N)}( T + (1/N) sum_n (Y_n/mu - Z_n) )      eq. (15)
//   Y_n  += mu (T - Z_n - E)                                      line 6
//   r_n   = max |T - Z_n - E|                                     line 8
// The state keeps D = T - E instead of E.  With h = T + m, m the mean above
// and theta = 1/(mu N): D = T where |h| <= theta and D = sgn(h) theta - m
// elsewhere, an exact rewrite of T - prox(h) that avoids subtracting two
// large numbers when |E| >> |T - E|.  Then T - Z_n - E = D - Z_n.
#include <math.h>

#include <algorithm>

#include "pasd_internal.hpp"

namespace pasd {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
template <typename S> struct V4;
template <> struct V4<float> { typedef f4v t; };
template <> struct V4<double> { typedef d4v t; };

template <typename S, int VEC>
__device__ __forceinline__ void loadv(const S* __restrict__ p, int64_t off, S out[VEC]) {
  if constexpr (VEC == 4) {
    typename V4<S>::t v = *reinterpret_cast<const typename V4<S>::t*>(p + off);
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = v[t];
  } else {
    out[0] = p[off];
  }
}

template <typename S, int VEC>
__device__ __forceinline__ void storev(S* __restrict__ p, int64_t off, const S in[VEC]) {
  if constexpr (VEC == 4) {
    typename V4<S>::t v;
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = in[t];
    *reinterpret_cast<typename V4<S>::t*>(p + off) = v;
  } else {
    p[off] = in[0];
  }
}

// Z_n at elements x0 .. x0+VEC-1 (all in one row of the last mode when VEC = 4).
template <typename S, int VEC>
__device__ __forceinline__ void recon(const Problem<S>& pb, int n, int64_t x0, S z[VEC]) {
  const ModeGeom& g = pb.g[n];
  const ModeBufs<S>& mb = pb.m[n];
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = S(0);
  if (g.B == 1) {
    const int64_t row = x0 / g.I;
    const int i = (int)(x0 - row * g.I);
    for (int r = 0; r < g.R; ++r) {
      const S pr = mb.P[(int64_t)r * g.J + row];
      S u[VEC];
      loadv<S, VEC>(mb.UfT, (int64_t)r * g.I + i, u);
#pragma unroll
      for (int t = 0; t < VEC; ++t) z[t] += u[t] * pr;
    }
  } else {
    const int64_t IB = (int64_t)g.I * g.B;
    const int64_t a = x0 / IB;
    const int64_t rem = x0 - a * IB;
    const int i = (int)(rem / g.B);
    const int64_t b = rem - (int64_t)i * g.B;
    const int64_t j = a * g.B + b;
    for (int r = 0; r < g.R; ++r) {
      const S u = mb.Uf[(int64_t)i * kRT + r];
      S pv[VEC];
      loadv<S, VEC>(mb.P, (int64_t)r * g.J + j, pv);
#pragma unroll
      for (int t = 0; t < VEC; ++t) z[t] += u * pv[t];
    }
  }
}

template <typename S>
__device__ __forceinline__ S nanmax(S a, S b) {
  return (b > a || b != b) ? b : a;
}

// Block-wide maximum of the per-thread residual maxima (blockDim = 256), one
// atomicMax per block and mode on slot blockIdx % kResSlots.  Max is exact, so
// the result does not depend on the order.  NaN propagates (its bit pattern
// exceeds every finite non-negative double).
template <int NN, typename S>
__device__ __forceinline__ void block_residual_max(DevScalars* sc, const S (&rmax)[NN], int lblk) {
  __shared__ double red[4][NN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    double r = (double)rmax[n];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r = nanmax(r, __shfl_xor(r, o, 64));
    if (lane == 0) red[wave][n] = r;
  }
  __syncthreads();
  if (threadIdx.x < NN) {
    const int n = threadIdx.x;
    const double r = nanmax(nanmax(red[0][n], red[1][n]), nanmax(red[2][n], red[3][n]));
    atomicMax(&sc->res_slots[n][lblk % kResSlots], (unsigned long long)__double_as_longlong(r));
  }
}

// Row view of the tensor for the fused pass: rows = numel / I_N of length I_N.
// For a mode n < N-1 the row index splits as row = (a * I_n + i_n) * Rb_n + rb
// with Rb_n = B_n / I_N, and the unfolding column is j = a * B_n + rb * I_N + i.
struct RowGeom {
  uint64_t IN;       // I_N
  uint64_t Rb[kMaxN];
};

// Z_n at the VEC elements starting at column i of `row`, with the rank loop
// unrolled to RP (P_n has zero rows up to kRT, U_n W_n zero columns), so that
// all loads of P_n and U_n W_n are independent and issue together.
template <typename S, int VEC, int RP, typename IT>
__device__ __forceinline__ void recon_row(const Problem<S>& pb, const RowGeom& rg, int n, bool last,
                                          IT row, IT i, S z[VEC]) {
  const ModeGeom& g = pb.g[n];
  const ModeBufs<S>& mb = pb.m[n];
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = S(0);
  if (last) {
    S pr[RP];
    S u[RP][VEC];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      pr[r] = mb.P[(int64_t)r * g.J + row];
      loadv<S, VEC>(mb.UfT + (int64_t)r * g.I, i, u[r]);
    }
#pragma unroll
    for (int r = 0; r < RP; ++r)
#pragma unroll
      for (int t = 0; t < VEC; ++t) z[t] += u[r][t] * pr[r];
  } else {
    const IT Rb = (IT)rg.Rb[n];
    const IT q1 = Rb == 1 ? row : row / Rb;
    const IT a = g.A == 1 ? IT(0) : q1 / (IT)g.I;
    const IT in = q1 - a * (IT)g.I;
    const IT j = a * (IT)g.B + (row - q1 * Rb) * (IT)rg.IN + i;
    S u[RP];
    S pv[RP][VEC];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      u[r] = mb.Uf[(int64_t)in * kRT + r];
      loadv<S, VEC>(mb.P + (int64_t)r * g.J, j, pv[r]);
    }
#pragma unroll
    for (int r = 0; r < RP; ++r)
#pragma unroll
      for (int t = 0; t < VEC; ++t) z[t] += u[r] * pv[r][t];
  }
}

// One problem's share of the fused pass: `nblk` blocks of which this is `lblk`.
template <typename S, int NN, int VEC, int RP, typename IT>
__device__ __forceinline__ void fused_body(const Problem<S>& pb, int lblk, int nblk) {
  RowGeom rg;
  rg.IN = (uint64_t)pb.g[NN - 1].I;
#pragma unroll
  for (int n = 0; n < NN - 1; ++n) rg.Rb[n] = (uint64_t)pb.g[n].B / rg.IN;
  const double mu_d = pb.sc->mu;
  const S mu = (S)mu_d;
  const S inv_mu = (S)(1.0 / mu_d);
  const S theta = (S)(1.0 / (mu_d * NN));
  const S invN = (S)(1.0 / NN);
  S rmax[NN];
#pragma unroll
  for (int n = 0; n < NN; ++n) rmax[n] = S(0);
  const IT nchunk = (IT)(pb.numel / VEC);
  const IT Q = (IT)(rg.IN / VEC);
  for (IT c = (IT)lblk * blockDim.x + threadIdx.x; c < nchunk; c += (IT)nblk * blockDim.x) {
    const IT row = c / Q;
    const IT i = (c - row * Q) * VEC;
    const IT x0 = c * VEC;
    S tv[VEC];
    loadv<S, VEC>(pb.T, x0, tv);
    S z[NN][VEC];
    S y[NN][VEC];
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      recon_row<S, VEC, RP, IT>(pb, rg, n, n == NN - 1, row, i, z[n]);
      loadv<S, VEC>(pb.m[n].Y, x0, y[n]);
    }
    S dv[VEC];
#pragma unroll
    for (int t = 0; t < VEC; ++t) {
      S s = S(0);
#pragma unroll
      for (int n = 0; n < NN; ++n) s += y[n][t] * inv_mu - z[n][t];
      const S m = s * invN;
      const S h = tv[t] + m;
      const S d = (fabs(h) <= theta) ? tv[t] : (copysign(theta, h) - m);
      dv[t] = d;
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        const S res = d - z[n][t];
        y[n][t] += mu * res;
        rmax[n] = nanmax(rmax[n], (S)fabs(res));
      }
    }
    storev<S, VEC>(pb.D, x0, dv);
#pragma unroll
    for (int n = 0; n < NN; ++n) storev<S, VEC>(pb.m[n].Y, x0, y[n]);
  }
  block_residual_max<NN>(pb.sc, rmax, lblk);
}

// The fused pass over a batch; each problem takes the vector path when its
// last dimension is a multiple of 4.
template <typename S, int NN, int RP, typename IT>
__global__ void __launch_bounds__(256) k_fused(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int lblk = blockIdx.x - bt.start[req];
  const int nblk = bt.start[req + 1] - bt.start[req];
  if (pb.vec4)
    fused_body<S, NN, 4, RP, IT>(pb, lblk, nblk);
  else
    fused_body<S, NN, 1, RP, IT>(pb, lblk, nblk);
}

// One wave: fold the residual slots (and clear them for the next iteration),
// then lane 0 applies Algorithm 1, lines 7-8.
template <typename S>
__global__ void __launch_bounds__(64) k_control(Batch<S> bt) {
  const Problem<S>& pb = *bt.p[blockIdx.x];
  DevScalars* sc = pb.sc;
  if (sc->done) return;
  __shared__ double res[kMaxN];
  const int lane = threadIdx.x;
  for (int n = 0; n < pb.N; ++n) {
    unsigned long long b = sc->res_slots[n][lane];
    sc->res_slots[n][lane] = 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long other = __shfl_xor(b, o, 64);
      b = other > b ? other : b;
    }
    if (lane == 0) res[n] = __longlong_as_double((long long)b);
  }
  if (lane != 0) return;
  bool conv = true, bad = false;
  for (int n = 0; n < pb.N; ++n) {
    const double r = res[n];
    sc->residual[n] = r;
    pb.hist[(int64_t)sc->k * pb.N + n] = r;
    if (!(r < pb.tol)) conv = false;
    if (!isfinite(r)) bad = true;
  }
  sc->mu = fmin(pb.rho * sc->mu, pb.mu_max);
  sc->k += 1;
  if (bad) {
    sc->done = 3;
  } else if (conv) {
    sc->converged = 1;
    sc->done = 1;
  } else if (sc->k >= pb.max_iter) {
    sc->done = 2;
  }
}

// Initialisation of Algorithm 1: E = 0 (D = T), Y_n = 0, U_n = eye(I_n, R_n).
template <typename S>
__global__ void __launch_bounds__(256) k_init_elem(Problem<S> pb) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < pb.numel;
       x += (int64_t)gridDim.x * blockDim.x) {
    pb.D[x] = pb.T[x];
    for (int n = 0; n < pb.N; ++n) pb.m[n].Y[x] = S(0);
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_init_small(Problem<S> pb, double mu0) {
  const int n = blockIdx.x;
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  for (int e = threadIdx.x; e < g.I * kRT; e += blockDim.x) {
    const int i = e / kRT, c = e - i * kRT;
    const double v = (i == c && c < g.R) ? 1.0 : 0.0;
    if (c < g.R) mb.U[(int64_t)i * g.R + c] = v;
    mb.Us[e] = (S)v;
  }
  if (n == 0 && threadIdx.x == 0) {
    DevScalars* sc = pb.sc;
    sc->mu = mu0;
    sc->k = 0;
    sc->done = 0;
    sc->converged = 0;
    for (int m = 0; m < kMaxN; ++m) {
      sc->residual[m] = 0.0;
      sc->rank[m] = 0;
      sc->eig_sweeps[m] = 0;
    }
  }
  if (n == 0)
    for (int e = threadIdx.x; e < kMaxN * kResSlots; e += blockDim.x)
      pb.sc->res_slots[e / kResSlots][e % kResSlots] = 0ull;
}

// X = sum_n alpha_n Z_n / sum_n alpha_n (output of Algorithm 1) and E = T - D.
template <typename S>
__global__ void __launch_bounds__(256) k_output(Problem<S> pb, S* X, S* E) {
  double wsum = 0;
  for (int n = 0; n < pb.N; ++n) wsum += pb.alpha[n];
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < pb.numel;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (X) {
      double acc = 0;
      for (int n = 0; n < pb.N; ++n) {
        S z[1];
        recon<S, 1>(pb, n, x, z);
        acc += pb.alpha[n] * (double)z[0];
      }
      X[x] = (S)(acc / wsum);
    }
    if (E) E[x] = pb.T[x] - pb.D[x];
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_component(Problem<S> pb, int n, S* Z) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < pb.numel;
       x += (int64_t)gridDim.x * blockDim.x) {
    S z[1];
    recon<S, 1>(pb, n, x, z);
    Z[x] = z[0];
  }
}

static int elem_grid(int64_t work) {
  int64_t b = (work + 255) / 256;
  if (b > 256 * 16) b = 256 * 16;
  if (b < 1) b = 1;
  return (int)b;
}

int fused_blocks(int64_t numel, bool vec4) { return elem_grid(vec4 ? numel / 4 : numel); }

template <typename S, int NN, int RP>
static void fused_idx(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int grid = make_batch(ls, b, [](const Problem<S>& p) { return p.fused_blocks; });
  bool big = false;
  for (int r = 0; r < ls.count; ++r) big = big || ls.host[r]->numel >= (int64_t(1) << 31);
  if (!big)
    hipLaunchKernelGGL((k_fused<S, NN, RP, uint32_t>), dim3(grid), dim3(256), 0, s, b);
  else  // tensors of 2^31 elements or more: 64-bit indexing, full rank tile
    hipLaunchKernelGGL((k_fused<S, NN, kRT, uint64_t>), dim3(grid), dim3(256), 0, s, b);
}

// The rank loop is unrolled to the largest R_n of the set rounded up to 4.
template <typename S, int NN>
static void fused_n(const LaunchSet<S>& ls, hipStream_t s) {
  int rmax = 1;
  for (int r = 0; r < ls.count; ++r)
    for (int n = 0; n < ls.host[r]->N; ++n) rmax = std::max(rmax, ls.host[r]->g[n].R);
  if (rmax <= 4)
    fused_idx<S, NN, 4>(ls, s);
  else if (rmax <= 8)
    fused_idx<S, NN, 8>(ls, s);
  else if (rmax <= 12)
    fused_idx<S, NN, 12>(ls, s);
  else
    fused_idx<S, NN, 16>(ls, s);
}

// All problems of a set have the same order N (the batch driver groups them).
template <typename S>
void launch_fused(const LaunchSet<S>& ls, hipStream_t s) {
  switch (ls.host[0]->N) {
    case 2: fused_n<S, 2>(ls, s); break;
    case 3: fused_n<S, 3>(ls, s); break;
    case 4: fused_n<S, 4>(ls, s); break;
    case 5: fused_n<S, 5>(ls, s); break;
    case 6: fused_n<S, 6>(ls, s); break;
    case 7: fused_n<S, 7>(ls, s); break;
    default: fused_n<S, 8>(ls, s); break;
  }
}

template <typename S>
void launch_control(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int grid = make_batch(ls, b, [](const Problem<S>&) { return 1; });
  hipLaunchKernelGGL(k_control<S>, dim3(grid), dim3(64), 0, s, b);
}

template <typename S>
void launch_init(const Problem<S>& p, double mu0, hipStream_t s) {
  hipLaunchKernelGGL(k_init_elem<S>, dim3(elem_grid(p.numel)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_init_small<S>, dim3(p.N), dim3(256), 0, s, p, mu0);
}

template <typename S>
void launch_output(const Problem<S>& p, S* X, S* E, hipStream_t s) {
  hipLaunchKernelGGL(k_output<S>, dim3(elem_grid(p.numel)), dim3(256), 0, s, p, X, E);
}

template <typename S>
void launch_component(const Problem<S>& p, int n, S* Z, hipStream_t s) {
  hipLaunchKernelGGL(k_component<S>, dim3(elem_grid(p.numel)), dim3(256), 0, s, p, n, Z);
}

#define INST(S)                                                              \
  template void launch_fused<S>(const LaunchSet<S>&, hipStream_t);           \
  template void launch_control<S>(const LaunchSet<S>&, hipStream_t);         \
  template void launch_init<S>(const Problem<S>&, double, hipStream_t);      \
  template void launch_output<S>(const Problem<S>&, S*, S*, hipStream_t);    \
  template void launch_component<S>(const Problem<S>&, int, S*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace pasd
