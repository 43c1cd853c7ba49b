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
#include <type_traits>

#include "pasd_internal.hpp"

namespace pasd {

// 16-byte vectors: 4 floats or 2 doubles per lane and access.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename S> struct VW;
template <> struct VW<float> { typedef f4v t; static constexpr int n = 4; };
template <> struct VW<double> { typedef d2v t; static constexpr int n = 2; };

// Z_n at element x (any layout), FP64 accumulation; used by the output passes.
template <typename S>
__device__ __forceinline__ double recon1(const Problem<S>& pb, int n, int64_t x) {
  const ModeGeom& g = pb.g[n];
  const ModeBufs<S>& mb = pb.m[n];
  double z = 0.0;
  const int64_t IB = (int64_t)g.I * g.B;
  const int64_t a = x / IB;
  const int64_t rem = x - a * IB;
  const int i = (int)(rem / g.B);
  const int64_t j = a * g.B + (rem - (int64_t)i * g.B);
  for (int r = 0; r < g.R; ++r)
    z = fma((double)mb.Uf[((int64_t)(r / kRT) * g.I + i) * kRT + r % kRT],
            (double)mb.P[(int64_t)r * g.J + j], z);
  return z;
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
  // entries 0..NN-2 are the residuals of the modes, entry NN-1 is max |D|
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
    const int row = n < NN - 1 ? n : kMaxN;
    atomicMax(&sc->res_slots[row][lblk % kResSlots], (unsigned long long)__double_as_longlong(r));
  }
}

// Accesses of the fused pass go through explicitly global pointers (no generic
// "flat" accesses, which also occupy the LDS/scalar wait counter) at a uniform
// base plus an element offset.  With a 32-bit index type the byte offset is a
// 32-bit value (the host takes that path only when every offset of the pass
// fits in 32 bits); otherwise it is 64-bit.
#define PASD_GLOBAL __attribute__((address_space(1)))

template <typename S, typename IT>
__device__ __forceinline__ uint64_t byte_off(IT idx) {
  if constexpr (sizeof(IT) == 4)
    return (uint32_t)(idx * (uint32_t)sizeof(S));
  else
    return (uint64_t)idx * sizeof(S);
}

template <typename S, int VEC, typename IT>
__device__ __forceinline__ void gload(const S* base, IT idx, S out[VEC]) {
  const PASD_GLOBAL char* p = (const PASD_GLOBAL char*)base + byte_off<S, IT>(idx);
  if constexpr (VEC > 1) {
    static_assert(VEC == VW<S>::n, "vector width");
    const typename VW<S>::t v = *(const PASD_GLOBAL typename VW<S>::t*)p;
#pragma unroll
    for (int t = 0; t < VEC; ++t) out[t] = v[t];
  } else {
    out[0] = *(const PASD_GLOBAL S*)p;
  }
}

// nt: non-temporal store (Problem::ntstore)
template <typename S, int VEC, typename IT>
__device__ __forceinline__ void gstore(S* base, IT idx, const S in[VEC], bool nt) {
  PASD_GLOBAL char* p = (PASD_GLOBAL char*)base + byte_off<S, IT>(idx);
  if constexpr (VEC > 1) {
    typename VW<S>::t v;
#pragma unroll
    for (int t = 0; t < VEC; ++t) v[t] = in[t];
    if (nt)
      __builtin_nontemporal_store(v, (PASD_GLOBAL typename VW<S>::t*)p);
    else
      *(PASD_GLOBAL typename VW<S>::t*)p = v;
  } else {
    *(PASD_GLOBAL S*)p = in[0];
  }
}

template <typename IT>
__device__ __forceinline__ IT div_fixed(IT n, IT d, FastDiv f) {
  if constexpr (sizeof(IT) == 4)
    return fastdiv(n, f);
  else
    return n / d;
}

// Running maximum of |v| kept as the bits of |v|: for non-negative IEEE values
// the integer order is the numeric order, and a NaN (any sign) compares above
// +inf, so a NaN residual survives the maximum.
template <typename E> struct AbsMax;
template <> struct AbsMax<float> {
  uint32_t b = 0;
  __device__ __forceinline__ void add(float v) {
    const uint32_t x = __float_as_uint(v) & 0x7fffffffu;
    b = x > b ? x : b;
  }
  __device__ __forceinline__ double get() const { return (double)__uint_as_float(b); }
};
template <> struct AbsMax<double> {
  uint64_t b = 0;
  __device__ __forceinline__ void add(double v) {
    const uint64_t x = (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
    b = x > b ? x : b;
  }
  __device__ __forceinline__ double get() const { return __longlong_as_double((long long)b); }
};

// What the fused pass needs of one problem, read once into registers before
// the first store (so that the compiler keeps it in scalar registers instead
// of re-reading it after every store to Y or D).
//
// Row view: rows = numel / I_N of length I_N.  For a mode n < N-1 the row index
// splits as row = (a * I_n + i_n) * Rb_n + rb with Rb_n = B_n / I_N, and the
// mode-n unfolding column of the element in column i of the row is
// j = a * B_n + rb * I_N + i.  For the last mode, i_N = i and j = row.
template <typename S, int NN, typename IT>
struct FusedView {
  const S* T;
  S* D;
  S* Y[NN];
  const S* P[NN];
  const S* F[NN];  // U_n W_n (rows of kRT) for n < N-1, its transpose for the last mode
  IT J[NN], I[NN], B[NN], Rb[NN];
  int NT[NN];      // rank tiles (the tile-looped rank path)
  IT IN, Q, nchunk;
  FastDiv fq, frb[NN], fi[NN];
  int nt;  // Problem::ntstore
};

template <typename S, int NN, int VEC, typename IT>
__device__ __forceinline__ FusedView<S, NN, IT> fused_view(const Problem<S>& pb) {
  FusedView<S, NN, IT> v;
  v.T = pb.T;
  v.D = pb.D;
  v.IN = (IT)pb.g[NN - 1].I;
  v.Q = v.IN / VEC;
  v.nchunk = (IT)(pb.numel / VEC);
  v.fq = pb.fd_q;
  v.nt = pb.ntstore;
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    v.Y[n] = pb.m[n].Y;
    v.P[n] = pb.m[n].P;
    v.F[n] = n < NN - 1 ? pb.m[n].Uf : pb.m[n].UfT;
    v.J[n] = (IT)pb.g[n].J;
    v.I[n] = (IT)pb.g[n].I;
    v.B[n] = (IT)pb.g[n].B;
    v.Rb[n] = (IT)(pb.g[n].B / pb.g[NN - 1].I);
    v.NT[n] = pb.g[n].T;
    v.frb[n] = pb.fd_rb[n];
    v.fi[n] = pb.fd_i[n];
  }
  return v;
}

// Z_n at the VEC elements starting at column i of `row`, accumulated in the
// state type, with the rank loop unrolled to RP (P_n has zero rows up to kRT
// and U_n W_n zero columns).  A scheduling barrier after the loads keeps them
// issued together: left alone, the compiler interleaves loads and FMAs to save
// registers and waits on each load in turn.
// RP = 0: ranks beyond one tile, a loop over the mode's T rank tiles with the
// tile's 16 ranks unrolled (U_n W_n tile-major: tile t of row in_n at
// (t I_n + in_n) kRT).
template <typename S, typename ZT, int NN, int VEC, typename IT>
__device__ __forceinline__ void recon_row_tiles(const FusedView<S, NN, IT>& v, int n, IT row, IT i,
                                                ZT z[VEC]) {
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = ZT(0);
  const int T = v.NT[n];
  if (n == NN - 1) {
    for (int tt = 0; tt < T; ++tt) {
      S pr[kRT];
      S u[kRT][VEC];
#pragma unroll
      for (int r = 0; r < kRT; ++r) {
        const IT rr = (IT)(tt * kRT + r);
        gload<S, 1, IT>(v.P[n], rr * v.J[n] + row, &pr[r]);
        gload<S, VEC, IT>(v.F[n], rr * v.IN + i, u[r]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < kRT; ++r)
#pragma unroll
        for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r][t], (ZT)pr[r], z[t]);
    }
  } else {
    const IT q1 = div_fixed<IT>(row, v.Rb[n], v.frb[n]);
    const IT a = n == 0 ? IT(0) : div_fixed<IT>(q1, v.I[n], v.fi[n]);  // A_0 = 1
    const IT in = q1 - a * v.I[n];
    const IT j = a * v.B[n] + (row - q1 * v.Rb[n]) * v.IN + i;
    constexpr int W = VW<S>::n;
    for (int tt = 0; tt < T; ++tt) {
      S u[kRT];
#pragma unroll
      for (int r = 0; r < kRT; r += W)
        gload<S, W, IT>(v.F[n], ((IT)tt * v.I[n] + in) * (IT)kRT + (IT)r, &u[r]);
      S pv[kRT][VEC];
#pragma unroll
      for (int r = 0; r < kRT; ++r)
        gload<S, VEC, IT>(v.P[n], (IT)(tt * kRT + r) * v.J[n] + j, pv[r]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < kRT; ++r)
#pragma unroll
        for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r], (ZT)pv[r][t], z[t]);
    }
  }
}

template <typename S, typename ZT, int NN, int VEC, int RP, typename IT>
__device__ __forceinline__ void recon_row(const FusedView<S, NN, IT>& v, int n, IT row, IT i,
                                          ZT z[VEC]) {
  if constexpr (RP == 0) {
    recon_row_tiles<S, ZT, NN, VEC, IT>(v, n, row, i, z);
  } else {
#pragma unroll
    for (int t = 0; t < VEC; ++t) z[t] = ZT(0);
    if (n == NN - 1) {
      S pr[RP];
      S u[RP][VEC];
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        gload<S, 1, IT>(v.P[n], (IT)r * v.J[n] + row, &pr[r]);
        gload<S, VEC, IT>(v.F[n], (IT)r * v.IN + i, u[r]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < RP; ++r)
#pragma unroll
        for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r][t], (ZT)pr[r], z[t]);
    } else {
      const IT q1 = div_fixed<IT>(row, v.Rb[n], v.frb[n]);
      const IT a = n == 0 ? IT(0) : div_fixed<IT>(q1, v.I[n], v.fi[n]);  // A_0 = 1
      const IT in = q1 - a * v.I[n];
      const IT j = a * v.B[n] + (row - q1 * v.Rb[n]) * v.IN + i;
      constexpr int W = VW<S>::n;  // U_n W_n rows are kRT long and 16-byte aligned
      // U_n W_f rows are kRT wide and zero beyond R: read whole 16-byte vectors
      constexpr int RU = (RP + W - 1) / W * W;
      S u[RU];
#pragma unroll
      for (int r = 0; r < RU; r += W) gload<S, W, IT>(v.F[n], in * (IT)kRT + (IT)r, &u[r]);
      S pv[RP][VEC];
#pragma unroll
      for (int r = 0; r < RP; ++r) gload<S, VEC, IT>(v.P[n], (IT)r * v.J[n] + j, pv[r]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < RP; ++r)
#pragma unroll
        for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r], (ZT)pv[r][t], z[t]);
    }
  }
}

// Merged modes (Problem::mmerge): the columns P_n[:, j .. j + VEC) of a
// chunk of a mode n < N-1, the loads recon_row issues for that mode.
template <typename S, int NN, int VEC, int RP, typename IT>
__device__ __forceinline__ void merged_cols(const FusedView<S, NN, IT>& v, int n, IT row, IT i,
                                            IT& in, S (&pv)[RP][VEC]) {
  const IT q1 = div_fixed<IT>(row, v.Rb[n], v.frb[n]);
  const IT a = n == 0 ? IT(0) : div_fixed<IT>(q1, v.I[n], v.fi[n]);  // A_0 = 1
  in = q1 - a * v.I[n];
  const IT j = a * v.B[n] + (row - q1 * v.Rb[n]) * v.IN + i;
#pragma unroll
  for (int r = 0; r < RP; ++r) gload<S, VEC, IT>(v.P[n], (IT)r * v.J[n] + j, pv[r]);
}

// recon_row of a merged mode, keeping the P_n columns for the GEMM-M sums.
template <typename S, typename ZT, int NN, int VEC, int RP, typename IT>
__device__ __forceinline__ void recon_row_keep(const FusedView<S, NN, IT>& v, int n, IT row, IT i,
                                               ZT z[VEC], S (&pv)[RP][VEC]) {
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = ZT(0);
  IT in;
  merged_cols<S, NN, VEC, RP, IT>(v, n, row, i, in, pv);
  constexpr int W = VW<S>::n;
  constexpr int RU = (RP + W - 1) / W * W;
  S u[RU];
#pragma unroll
  for (int r = 0; r < RU; r += W) gload<S, W, IT>(v.F[n], in * (IT)kRT + (IT)r, &u[r]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < RP; ++r)
#pragma unroll
    for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r], (ZT)pv[r][t], z[t]);
}

// recon_row_keep with the mode's U_n W_f row already in registers (a merged
// mode's index i_n is the same for every chunk of a block).
template <typename S, typename ZT, int NN, int VEC, int RP, int RU, typename IT>
__device__ __forceinline__ void recon_keep_u(const FusedView<S, NN, IT>& v, int n, IT row, IT i,
                                             ZT z[VEC], S (&pv)[RP][VEC], const S (&u)[RU]) {
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = ZT(0);
  IT in;
  merged_cols<S, NN, VEC, RP, IT>(v, n, row, i, in, pv);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < RP; ++r)
#pragma unroll
    for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r], (ZT)pv[r][t], z[t]);
}

// recon_row of the last mode with its (U W)^T columns i .. i + VEC already in
// registers.
template <typename S, typename ZT, int NN, int VEC, int RP, typename IT>
__device__ __forceinline__ void recon_last_u(const FusedView<S, NN, IT>& v, IT row, ZT z[VEC],
                                             const S (&u)[RP][VEC]) {
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = ZT(0);
  S pr[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) gload<S, 1, IT>(v.P[NN - 1], (IT)r * v.J[NN - 1] + row, &pr[r]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < RP; ++r)
#pragma unroll
    for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r][t], (ZT)pr[r], z[t]);
}

// GEMM-M of the next iteration for one merged mode at one chunk:
// acc[r] += G(x) P_n[r, j(x)] with G = D + Y_n / mu (state type, one fused
// multiply-add, as the GEMM-M kernels form it) and FP64 products and sums.
template <typename S, int VEC, int RP>
__device__ __forceinline__ void macc_add(double (&acc)[RP], const S (&pv)[RP][VEC],
                                         const S (&d)[VEC], const S (&y)[VEC], S inv_mu) {
#pragma unroll
  for (int t = 0; t < VEC; ++t) {
    const S g = fma(y[t], inv_mu, d[t]);
#pragma unroll
    for (int r = 0; r < RP; ++r) acc[r] = fma((double)g, (double)pv[r][t], acc[r]);
  }
}

// The block's partial sums of the merged modes' M_n rows (blockDim = 256,
// fixed-order reduction: wave butterflies, then the four waves in order),
// written to Mf_n[b][0 .. RP).
template <typename S, int MM, int RP>
__device__ __forceinline__ void macc_store(const Problem<S>& pb, const double (&acc)[MM][RP],
                                           int b) {
  __shared__ double red[4][MM * RP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int n = 0; n < MM; ++n)
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      double v = acc[n][r];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[wave][n * RP + r] = v;
    }
  __syncthreads();
  if (threadIdx.x < MM * RP) {
    const int n = threadIdx.x / RP, r = threadIdx.x % RP;
    const double v = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                     red[3][threadIdx.x];
    pb.m[n].Mf[(int64_t)b * kRT + r] = v;
  }
}

// Z_n from a factor row staged in LDS: u (U_n W_f row, or the last mode's P
// column) read as 16-byte vectors, times the VEC columns pv already loaded.
template <typename S, typename ZT, int VEC, int RP, int RU>
__device__ __forceinline__ void recon_lds(const S* u_lds, const S (&pv)[RP][VEC], ZT z[VEC]) {
  constexpr int W = VW<S>::n;
  S u[RU];
#pragma unroll
  for (int r = 0; r < RU; r += W) {
    const typename VW<S>::t x = *reinterpret_cast<const typename VW<S>::t*>(u_lds + r);
#pragma unroll
    for (int t = 0; t < W; ++t) u[r + t] = x[t];
  }
#pragma unroll
  for (int t = 0; t < VEC; ++t) z[t] = ZT(0);
#pragma unroll
  for (int r = 0; r < RP; ++r)
#pragma unroll
    for (int t = 0; t < VEC; ++t) z[t] = fma((ZT)u[r], (ZT)pv[r][t], z[t]);
}

// Rows staged per block for the order-4 merged pass (mode 2's U W rows and the
// last mode's P columns of the block's rows).
constexpr int kStageRows = 128;

// x + x(lane ^ D) for D = 16 or 32, the same in both lanes: the gfx950 row
// swaps (v_permlane16_swap / v_permlane32_swap on two copies of x leave the
// even and the odd half of each pair of rows, or of the wave, in the two
// results), added even half first.
template <int D>
__device__ __forceinline__ double swap_sum(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)(b >> 32);
  unsigned l0, l1, h0, h1;
  if constexpr (D == 16) {
    const auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    l0 = L[0], l1 = L[1], h0 = H[0], h1 = H[1];
  } else {
    const auto L = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto H = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    l0 = L[0], l1 = L[1], h0 = H[0], h1 = H[1];
  }
  return __longlong_as_double(((long long)h0 << 32) | l0) +
         __longlong_as_double(((long long)h1 << 32) | l1);
}

// Sum of w over the Q aligned lanes of a row group (Q a power of two, at
// most 64), left in every lane of the group: DPP exchanges within quads (lanes
// i^1, i^2), the mirror images within 8 and 16 lanes, then lanes i^16 and
// i^32 by row swaps.  Every lane adds the same two values at each step (a + b
// and b + a round alike), so the order is fixed.
template <int NT>
__device__ __forceinline__ void group_sum(double (&w)[NT], uint32_t Q) {
  double t[NT];
  if (Q > 1) {
#pragma unroll
    for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppXor1>(w[e]);
#pragma unroll
    for (int e = 0; e < NT; ++e) w[e] += t[e];
  }
  if (Q > 2) {
#pragma unroll
    for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppXor2>(w[e]);
#pragma unroll
    for (int e = 0; e < NT; ++e) w[e] += t[e];
  }
  if (Q > 4) {
#pragma unroll
    for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppHalfMirror>(w[e]);
#pragma unroll
    for (int e = 0; e < NT; ++e) w[e] += t[e];
  }
  if (Q > 8) {
#pragma unroll
    for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppMirror>(w[e]);
#pragma unroll
    for (int e = 0; e < NT; ++e) w[e] += t[e];
  }
  if (Q > 16) {
#pragma unroll
    for (int e = 0; e < NT; ++e) w[e] = swap_sum<16>(w[e]);
  }
  if (Q > 32) {
#pragma unroll
    for (int e = 0; e < NT; ++e) w[e] = swap_sum<32>(w[e]);
  }
}

// The fast modes' GEMM-M terms of one chunk (Problem::mfull), with
// G_n = D + Y_n / mu formed as in the GEMM-M kernels and FP64 products: the
// last mode's go to the thread's own sums for its columns (acc3, P_3 column
// p3 of this row), mode 2's to w, this chunk's share of its row's sum over the
// thread's columns (P_2 columns p2, the same for every chunk of the thread).
template <typename S, int VEC, int RP>
__device__ __forceinline__ void fast_acc(double (&acc3)[VEC][RP], double (&w)[RP],
                                         const S (&p2)[RP][VEC], const S (&p3)[RP],
                                         const S (&d)[VEC], const S (&y2)[VEC],
                                         const S (&y3)[VEC], S inv_mu) {
#pragma unroll
  for (int t = 0; t < VEC; ++t) {
    const S g3 = fma(y3[t], inv_mu, d[t]);
#pragma unroll
    for (int r = 0; r < RP; ++r) acc3[t][r] = fma((double)g3, (double)p3[r], acc3[t][r]);
  }
#pragma unroll
  for (int r = 0; r < RP; ++r) w[r] = 0.0;
#pragma unroll
  for (int t = 0; t < VEC; ++t) {
    const S g2 = fma(y2[t], inv_mu, d[t]);
#pragma unroll
    for (int r = 0; r < RP; ++r) w[r] = fma((double)g2, (double)p2[r][t], w[r]);
  }
}

// Block end of the fast modes (Problem::mfull; blockDim = 256): the block's
// I_2 x R_2 partial of M_2 (its rows' sums m2[k][r] for i_2 = i2a + k, k <
// nrows, zero elsewhere) and I_3 x R_3 partial of M_3, which holds for column
// i_3 = VEC cq + t the sum over the threads cq, cq + Q, ... of their acc3[t]:
// first within each wave by lane butterflies over the lanes of equal column
// (xor Q, 2Q, ... below 64), then over the four waves in order.  (Writing each
// row's sums to global memory from inside the sweep was measured slower: the
// stores hold up the waits for the next chunk's loads.)
template <typename S, int NN, int VEC, int RP>
__device__ __forceinline__ void fast_store(const Problem<S>& pb, int lblk, double (&acc3)[VEC][RP],
                                           const double* m2, uint32_t i2a, uint32_t nrows,
                                           uint32_t Q) {
  constexpr int NV = VEC * RP;
  __shared__ double red3[4][64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (uint32_t o = Q; o < 64; o <<= 1) {
#pragma unroll
    for (int t = 0; t < VEC; ++t)
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const double x = acc3[t][r];
        acc3[t][r] = o == 16 ? swap_sum<16>(x) : o == 32 ? swap_sum<32>(x)
                                               : x + __shfl_xor(x, (int)o, 64);
      }
  }
  if ((uint32_t)lane < Q) {
#pragma unroll
    for (int t = 0; t < VEC; ++t)
#pragma unroll
      for (int r = 0; r < RP; ++r) red3[wave][lane][t * RP + r] = acc3[t][r];
  }
  __syncthreads();
  {
    const int R2 = pb.g[NN - 2].R;
    const uint32_t ne = (uint32_t)pb.g[NN - 2].I * R2;
    double* q2 = pb.m[NN - 2].Mq + (int64_t)lblk * ne;
    for (uint32_t e = threadIdx.x; e < ne; e += blockDim.x) {
      const uint32_t i2 = e / R2, r = e - i2 * R2;
      q2[e] = (i2 >= i2a && i2 - i2a < nrows) ? m2[(i2 - i2a) * RP + r] : 0.0;
    }
  }
  const int R3 = pb.g[NN - 1].R;
  double* q3 = pb.m[NN - 1].Mq + (int64_t)lblk * pb.g[NN - 1].I * R3;
  for (uint32_t e = threadIdx.x; e < Q * NV; e += blockDim.x) {
    const uint32_t cq = e / NV, k = e - cq * NV;
    const uint32_t t = k / RP, r = k - t * RP;
    if ((int)r >= R3) continue;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += red3[w][cq][k];  // every wave holds one sum per column
    q3[(cq * VEC + t) * R3 + r] = sum;
  }
}

// One problem's share of the fused pass: `nblk` blocks of which this is `lblk`.
// The arithmetic is in the state type: every quantity is formed with one
// rounding from stored state-type values (D - Z_n of two nearby values is
// exact, Y_n + mu (D - Z_n) is one fused multiply-add), so wider registers would
// change the stored iterate only through the rounding of mu.  The residual is
// taken from the stored D.
template <typename S, int NN, int VEC, int RP, typename IT, bool SPLIT1, int MM>
__device__ __forceinline__ void fused_body(const Problem<S>& pb, int lblk, int nblk, bool xcd_split) {
  // Accumulation type of Z_n and type of the elementwise arithmetic.  Both are
  // the state type: wider registers were measured to leave FP32 convergence
  // (iteration counts, converged fraction) unchanged and cost 5-10% here.
  typedef S ZT;
  typedef S ET;
  const FusedView<S, NN, IT> v = fused_view<S, NN, VEC, IT>(pb);
  const double mu_d = pb.sc->mu;
  const ET mu = (ET)mu_d;
  const ET inv_mu = (ET)(1.0 / mu_d);
  const ET theta = (ET)(1.0 / (mu_d * NN));
  const ET invN = (ET)(1.0 / NN);
  // the penalty of the next iteration, as the control kernel forms it, for
  // the merged modes' G = D + Y_n / mu
  const S inv_mu_next = (S)(1.0 / fmin(pb.rho * mu_d, pb.mu_max));
  AbsMax<ET> rmax[NN + 1];  // residual of every mode, then max |D|
  // Blocks are dealt to the 8 XCDs in turn (block b to XCD b mod 8).  When the
  // problem's blocks split evenly, the blocks of one XCD sweep (grid-stride)
  // one contiguous eighth of the tensor: the P_n columns a region needs are
  // fetched into one XCD's L2 instead of all eight, and each XCD's accesses
  // stay in one compact front.
  // With SPLIT1 (32-bit offsets only) XCD x enumerates e over the segments
  // of its mode-1 eighth: chunk = (e / f_seg) f_cp0 + x f_seg + e mod f_seg.
  IT c0 = 0, c1 = v.nchunk, first = (IT)lblk * blockDim.x, step = (IT)nblk * blockDim.x;
  IT seg_base = 0;
  // merged modes: block lblk sweeps its own mcb consecutive chunks
  double macc[MM > 0 ? MM : 1][RP > 0 ? RP : 1];
  // The U_n W_f rows of the merged modes are the same for the whole block
  // (its chunks lie in one slab of each), and when the row length in chunks
  // divides the block's start and stride, so are the last mode's columns for
  // all chunks of a thread: both are loaded once, before the sweep (64^4
  // FP64: 374 -> 350 us).  With an FP32 state, keeping the last mode's
  // columns was measured slower (173 -> 189 us; the compiler then holds every
  // load of a chunk before the first product), the merged rows alone faster
  // (169 us).
  constexpr bool kHoistU = MM > 0;
  constexpr bool kHoistLast = MM > 0 && sizeof(S) == 8;
  constexpr int RPk = RP > 0 ? RP : 1;
  constexpr int RUk = (RPk + VW<S>::n - 1) / VW<S>::n * VW<S>::n;
  S um[MM > 0 ? MM : 1][RUk];
  S ul[RPk][VEC];
  bool keep_last = false;
  // Order-4 merged blocks with an FP64 state stage mode 2's U W rows and the
  // last mode's P columns for their rows (at most kStageRows) in LDS, once per
  // block, in place of 9 global loads per chunk (64^4 R_n = 6: 350 -> 326 us;
  // with an FP32 state it gained nothing).  P_n and U_n W_f have zero rows /
  // columns up to kRT, so the padded reads stay in bounds.
  constexpr bool kStage = MM > 0 && NN == 4 && RP > 0 && sizeof(S) == 8;
  __shared__ __align__(16) S st_f[kStage ? kStageRows : 1][RUk];
  __shared__ __align__(16) S st_p[kStage ? kStageRows : 1][RUk];
  bool staged = false;
  IT st_row0 = 0;
  // with the last mode's columns fixed per thread, mode 2's P columns are too
  // (j_2 runs over (i_0, i_1, i_3), and i_0, i_1 are the block's); at rank 8
  // keeping them pushed the pass past 256 registers (one wave per SIMD, 64^4:
  // 364 -> 447 us) and they are loaded per chunk
  constexpr bool kHoistP2 = kStage && RP != 8;
  S p2k[kHoistP2 ? RPk : 1][VEC];
  // the fast modes' GEMM-M in the pass (Problem::mfull, ranks up to 6, the
  // 16-byte vector path)
  constexpr bool kFull = kHoistP2 && RP <= 6 && VEC == VW<S>::n;
  bool mfull = false;
  double acc3[kFull ? VEC : 1][kFull ? RPk : 1];
  __shared__ double st_m2[kFull ? kStageRows : 1][kFull ? RPk : 1];
  uint32_t st_i2a = 0, st_nrows = 0;
  if constexpr (MM > 0) {
#pragma unroll
    for (int n = 0; n < MM; ++n)
#pragma unroll
      for (int r = 0; r < RP; ++r) macc[n][r] = 0.0;
    c0 = (IT)lblk * (IT)pb.mcb;
    c1 = c0 + (IT)pb.mcb;
    first = 0;
    step = blockDim.x;
    if constexpr (kFull) {
#pragma unroll
      for (int t = 0; t < VEC; ++t)
#pragma unroll
        for (int r = 0; r < RPk; ++r) acc3[t][r] = 0.0;
    }
    const IT row0 = div_fixed<IT>(c0, v.Q, v.fq);
#pragma unroll
    for (int n = 0; n < (kHoistU ? MM : 0); ++n) {
      const IT q1 = div_fixed<IT>(row0, v.Rb[n], v.frb[n]);
      const IT a = n == 0 ? IT(0) : div_fixed<IT>(q1, v.I[n], v.fi[n]);
      const IT in = q1 - a * v.I[n];
#pragma unroll
      for (int r = 0; r < RUk; r += VW<S>::n)
        gload<S, VW<S>::n, IT>(v.F[n], in * (IT)kRT + (IT)r, &um[n][r]);
    }
    keep_last = kHoistLast && ((IT)blockDim.x % v.Q) == 0 && ((IT)pb.mcb % v.Q) == 0;
    if (keep_last) {
      const IT i0 = ((IT)threadIdx.x % v.Q) * VEC;
#pragma unroll
      for (int r = 0; r < RPk; ++r) gload<S, VEC, IT>(v.F[NN - 1], (IT)r * v.IN + i0, ul[r]);
    }
    if constexpr (kStage) {
      // the block's rows row0 .. row0 + nrows - 1: mode NN-2's U W rows at
      // their indices i_{NN-2} and the last mode's P columns at the rows
      st_row0 = row0;
      const IT nrows = div_fixed<IT>(c1 - 1, v.Q, v.fq) - row0 + 1;
      staged = nrows <= (IT)kStageRows;
      if (staged) {
        constexpr int n2 = NN - 2;
        for (IT e = threadIdx.x; e < nrows * (IT)RUk; e += blockDim.x) {
          const IT k = e / (IT)RUk, r = e - k * (IT)RUk;
          const IT row = row0 + k;
          const IT q1 = div_fixed<IT>(row, v.Rb[n2], v.frb[n2]);
          const IT a = div_fixed<IT>(q1, v.I[n2], v.fi[n2]);
          const IT in = q1 - a * v.I[n2];
          S f, pc;
          gload<S, 1, IT>(v.F[n2], in * (IT)kRT + r, &f);
          gload<S, 1, IT>(v.P[NN - 1], r * v.J[NN - 1] + row, &pc);
          st_f[k][r] = f;
          st_p[k][r] = pc;
        }
        if constexpr (kHoistP2) {
          if (keep_last) {
            IT in;
            merged_cols<S, NN, VEC, RPk, IT>(v, NN - 2, row0, ((IT)threadIdx.x % v.Q) * VEC, in,
                                             p2k);
            st_i2a = (uint32_t)in;
            st_nrows = (uint32_t)nrows;
          }
        }
      }
      // the host sets mfull only where both hold
      mfull = kFull && pb.mfull && staged && keep_last;
      __syncthreads();
    }
  } else if (xcd_split) {
    const int x = lblk % kXcds;
    first = (IT)(lblk / kXcds) * blockDim.x;
    step = (IT)(nblk / kXcds) * blockDim.x;
    if constexpr (SPLIT1) {
      c1 = v.nchunk / kXcds;  // every XCD enumerates an equal share
      seg_base = (IT)x * (IT)pb.f_seg;
    } else {
      const IT per = (v.nchunk + kXcds - 1) / kXcds;
      c0 = (IT)x * per;
      c1 = c0 + per < v.nchunk ? c0 + per : v.nchunk;
    }
  }
  for (IT e = c0 + first + threadIdx.x; e < c1; e += step) {
    IT c = e;
    if constexpr (SPLIT1) {
      const IT sg = (IT)fastdiv((uint32_t)e, pb.fd_seg);
      c = sg * (IT)pb.f_cp0 + seg_base + (e - sg * (IT)pb.f_seg);
    }
    const IT row = div_fixed<IT>(c, v.Q, v.fq);
    const IT i = (c - row * v.Q) * VEC;
    const IT x0 = c * VEC;
    S tv[VEC];
    gload<S, VEC, IT>(v.T, x0, tv);
    ZT z[NN][VEC];
    S y[NN][VEC];
    // the streamed operands first: the first mode's wait then covers their
    // HBM round trip and every later mode waits only for its own (cached)
    // factor loads
#pragma unroll
    for (int n = 0; n < NN; ++n) gload<S, VEC, IT>(v.Y[n], x0, y[n]);
    S pk[MM > 0 ? MM : 1][RP > 0 ? RP : 1][VEC];
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      if constexpr (MM > 0) {
        if (n < MM) {
          if constexpr (kHoistU)
            recon_keep_u<S, ZT, NN, VEC, RP, RUk, IT>(v, n, row, i, z[n], pk[n < MM ? n : 0],
                                                      um[n < MM ? n : 0]);
          else
            recon_row_keep<S, ZT, NN, VEC, RP, IT>(v, n, row, i, z[n], pk[n < MM ? n : 0]);
          continue;
        }
        if constexpr (kStage) {
          if (staged && n == NN - 2) {
            bool done_n = false;
            if constexpr (kHoistP2) {
              if (keep_last) {
                recon_lds<S, ZT, VEC, RPk, RUk>(&st_f[row - st_row0][0], p2k, z[n]);
                done_n = true;
              }
            }
            if (!done_n) {
              S pv[RPk][VEC];
              IT in;
              merged_cols<S, NN, VEC, RPk, IT>(v, n, row, i, in, pv);
              __builtin_amdgcn_sched_barrier(0);
              recon_lds<S, ZT, VEC, RPk, RUk>(&st_f[row - st_row0][0], pv, z[n]);
            }
            continue;
          }
          if (staged && n == NN - 1 && keep_last) {
            S pr[RUk];
#pragma unroll
            for (int r = 0; r < RUk; r += VW<S>::n) {
              const typename VW<S>::t x =
                  *reinterpret_cast<const typename VW<S>::t*>(&st_p[row - st_row0][r]);
#pragma unroll
              for (int t = 0; t < VW<S>::n; ++t) pr[r + t] = x[t];
            }
#pragma unroll
            for (int t = 0; t < VEC; ++t) z[n][t] = ZT(0);
#pragma unroll
            for (int r = 0; r < RPk; ++r)
#pragma unroll
              for (int t = 0; t < VEC; ++t) z[n][t] = fma((ZT)ul[r][t], (ZT)pr[r], z[n][t]);
            continue;
          }
        }
        if (n == NN - 1 && keep_last) {
          recon_last_u<S, ZT, NN, VEC, RPk, IT>(v, row, z[n], ul);
          continue;
        }
      }
      recon_row<S, ZT, NN, VEC, RP, IT>(v, n, row, i, z[n]);
    }
    S dv[VEC];
#pragma unroll
    for (int t = 0; t < VEC; ++t) {
      ET sum = ET(0);
#pragma unroll
      for (int n = 0; n < NN; ++n) sum += (ET)y[n][t] * inv_mu - (ET)z[n][t];
      const ET m = sum * invN;
      const ET tt = (ET)tv[t];
      const ET h = tt + m;
      dv[t] = (S)((fabs(h) <= theta) ? tt : (copysign(theta, h) - m));
      const ET d = (ET)dv[t];
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        const ET res = d - (ET)z[n][t];
        y[n][t] = (S)fma(mu, res, (ET)y[n][t]);
        rmax[n].add(res);
      }
      rmax[NN].add(d);
    }
    gstore<S, VEC, IT>(v.D, x0, dv, v.nt != 0);
#pragma unroll
    for (int n = 0; n < NN; ++n) gstore<S, VEC, IT>(v.Y[n], x0, y[n], v.nt != 0);
    if constexpr (MM > 0) {
#pragma unroll
      for (int n = 0; n < MM; ++n) macc_add<S, VEC, RP>(macc[n], pk[n], dv, y[n], inv_mu_next);
    }
    if constexpr (kFull) {
      if (mfull) {
        const IT kr = row - st_row0;
        S p3[RPk];
#pragma unroll
        for (int r = 0; r < RPk; ++r) p3[r] = st_p[kr][r];
        double w[RPk];
        fast_acc<S, VEC, RPk>(acc3, w, p2k, p3, dv, y[NN - 2], y[NN - 1], inv_mu_next);
        group_sum<RPk>(w, (uint32_t)v.Q);
        if ((IT)threadIdx.x % v.Q == 0) {
#pragma unroll
          for (int r = 0; r < RPk; ++r) st_m2[kr][r] = w[r];
        }
      }
    }
  }
  if constexpr (MM > 0) macc_store<S, MM, RP>(pb, macc, lblk);
  if constexpr (kFull) {
    if (mfull)
      fast_store<S, NN, VEC, RPk>(pb, lblk, acc3, &st_m2[0][0], st_i2a, st_nrows, (uint32_t)v.Q);
  }
  double r[NN + 1];
#pragma unroll
  for (int n = 0; n <= NN; ++n) r[n] = rmax[n].get();
  block_residual_max<NN + 1>(pb.sc, r, lblk);
}

// The fused pass over a batch; each problem takes the 16-byte vector path when
// its last dimension is a multiple of the vector width.
template <typename S, int NN, int RP, typename IT, bool SPLIT1, int MM>
__global__ void __launch_bounds__(256) k_fused(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int s0 = bt.start[req];
  const int nblk = bt.start[req + 1] - s0;
  const int lblk = blockIdx.x - s0;
  const bool xcd_split = nblk % kXcds == 0 && s0 % kXcds == 0;
  if constexpr (SPLIT1) {
    // launched only for one problem with fsplit1 set and a grid of whole
    // XCD rounds (a separate instantiation keeps the other's registers low)
    if (pb.vecw)
      fused_body<S, NN, VW<S>::n, RP, IT, true, 0>(pb, lblk, nblk, true);
    else
      fused_body<S, NN, 1, RP, IT, true, 0>(pb, lblk, nblk, true);
  } else {
    if (pb.vecw)
      fused_body<S, NN, VW<S>::n, RP, IT, false, MM>(pb, lblk, nblk, xcd_split);
    else
      fused_body<S, NN, 1, RP, IT, false, MM>(pb, lblk, nblk, xcd_split);
  }
}

// The merged modes' GEMM-M partials recomputed from the stored D, Y_n and
// P_n (after a checkpoint import, which restores the iterate but not these
// sums): the fused pass's traversal, loads and arithmetic, so the partials
// equal those the pass itself would have written.
template <typename S, int NN, int VEC, int RP, int MM>
__device__ __forceinline__ void mrefresh_body(const Problem<S>& pb, int lblk) {
  typedef uint32_t IT;
  const FusedView<S, NN, IT> v = fused_view<S, NN, VEC, IT>(pb);
  const S inv_mu = (S)(1.0 / pb.sc->mu);
  double macc[MM][RP];
#pragma unroll
  for (int n = 0; n < MM; ++n)
#pragma unroll
    for (int r = 0; r < RP; ++r) macc[n][r] = 0.0;
  const IT c0 = (IT)lblk * (IT)pb.mcb, c1 = c0 + (IT)pb.mcb;
  // the fast modes (Problem::mfull): the pass's P_2 columns, sums and order
  constexpr bool kFull = sizeof(S) == 8 && NN == 4 && RP <= 6 && VEC == VW<S>::n;
  const bool mfull = kFull && pb.mfull;
  double acc3[kFull ? VEC : 1][kFull ? RP : 1];
  S p2k[kFull ? RP : 1][VEC];
  __shared__ double st_m2[kFull ? kStageRows : 1][kFull ? RP : 1];
  const IT row0 = div_fixed<IT>(c0, v.Q, v.fq);
  uint32_t i2a = 0;
  if constexpr (kFull) {
    if (mfull) {
#pragma unroll
      for (int t = 0; t < VEC; ++t)
#pragma unroll
        for (int r = 0; r < RP; ++r) acc3[t][r] = 0.0;
      IT in;
      merged_cols<S, NN, VEC, RP, IT>(v, NN - 2, row0, ((IT)threadIdx.x % v.Q) * VEC, in, p2k);
      i2a = (uint32_t)in;
    }
  }
  for (IT c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const IT row = div_fixed<IT>(c, v.Q, v.fq);
    const IT i = (c - row * v.Q) * VEC;
    const IT x0 = c * VEC;
    S dv[VEC];
    gload<S, VEC, IT>(v.D, x0, dv);
    S y[MM][VEC];
    S pv[MM][RP][VEC];
#pragma unroll
    for (int n = 0; n < MM; ++n) {
      gload<S, VEC, IT>(v.Y[n], x0, y[n]);
      IT in;
      merged_cols<S, NN, VEC, RP, IT>(v, n, row, i, in, pv[n]);
    }
#pragma unroll
    for (int n = 0; n < MM; ++n) macc_add<S, VEC, RP>(macc[n], pv[n], dv, y[n], inv_mu);
    if constexpr (kFull) {
      if (mfull) {
        S y2[VEC], y3[VEC], p3[RP];
        gload<S, VEC, IT>(v.Y[NN - 2], x0, y2);
        gload<S, VEC, IT>(v.Y[NN - 1], x0, y3);
#pragma unroll
        for (int r = 0; r < RP; ++r) gload<S, 1, IT>(v.P[NN - 1], (IT)r * v.J[NN - 1] + row, &p3[r]);
        double w[RP];
        fast_acc<S, VEC, RP>(acc3, w, p2k, p3, dv, y2, y3, inv_mu);
        group_sum<RP>(w, (uint32_t)v.Q);
        if ((IT)threadIdx.x % v.Q == 0) {
#pragma unroll
          for (int r = 0; r < RP; ++r) st_m2[row - row0][r] = w[r];
        }
      }
    }
  }
  macc_store<S, MM, RP>(pb, macc, lblk);
  if constexpr (kFull) {
    if (mfull)
      fast_store<S, NN, VEC, RP>(pb, lblk, acc3, &st_m2[0][0], i2a, (uint32_t)(pb.mcb / v.Q),
                                 (uint32_t)v.Q);
  }
}

template <typename S, int NN, int RP, int MM>
__global__ void __launch_bounds__(256) k_mrefresh(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  const int lblk = blockIdx.x - bt.start[req];
  if (pb.vecw)
    mrefresh_body<S, NN, VW<S>::n, RP, MM>(pb, lblk);
  else
    mrefresh_body<S, NN, 1, RP, MM>(pb, lblk);
}

// One wave: fold the residual slots (and clear them for the next iteration),
// then lane 0 applies Algorithm 1, lines 7-8.
template <typename S>
__global__ void __launch_bounds__(64) k_control(Batch<S> bt) {
  const Problem<S>& pb = *bt.p[blockIdx.x];
  DevScalars* sc = pb.sc;
  if (sc->done) return;
  __shared__ double res_row[kMaxN + 1];  // folded slot rows; row kMaxN is max |D|
  __shared__ double res[kMaxN + 1];
  const int lane = threadIdx.x;
  // every row's slots are read before any is cleared, so the loads overlap
  unsigned long long b[kMaxN + 1];
#pragma unroll
  for (int r = 0; r <= kMaxN; ++r) b[r] = sc->res_slots[r][lane];
#pragma unroll
  for (int r = 0; r <= kMaxN; ++r) sc->res_slots[r][lane] = 0ull;
#pragma unroll
  for (int r = 0; r <= kMaxN; ++r) {
    if (r < pb.N || r == kMaxN) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(b[r], o, 64);
        b[r] = other > b[r] ? other : b[r];
      }
      if (lane == 0) res_row[r] = __longlong_as_double((long long)b[r]);
    }
  }
  if (lane != 0) return;
  for (int n = 0; n <= pb.N; ++n) res[n] = res_row[n < pb.N ? n : kMaxN];
  // Stopping test of Algorithm 1 (line 8): converged when every residual is
  // strictly below tol.  A rounded state cannot certify residuals below the
  // rounding of its own values: the N copies Z_n are rebuilt from different
  // rounded factors and disagree by a few units of the last place of |D|.
  // When every residual is below that level, c u max|D| with u the unit
  // roundoff of the state, but not below tol, the solve stops as "at the
  // precision floor" (done = 4, converged stays 0) unless the caller asked to
  // run on.  For an FP32 state c u = 16 * 2^-24: Z_n sums R_n rank terms
  // rounded in FP32, and where the data's magnitude makes the floor bind
  // (values up to 255) the residual levels off at 8-12 u max|D| (measured at
  // R_n = 16 and 40).  The split-BF16 GEMM operands carry FP32 accuracy, so
  // that mode shares the FP32 level; FP64 uses 8 * 2^-53.
  const double cu = sizeof(S) == 4 ? 9.5367431640625e-07 : 8.0 * 1.1102230246251565e-16;
  const double dmax = res[pb.N];
  const double floor_lvl = pb.tol > 0.0 ? fmax(pb.tol, cu * dmax) : 0.0;  // tol 0: never stop
  sc->dmax = dmax;
  sc->tol_eff = floor_lvl;
  bool conv = pb.tol > 0.0, at_floor = pb.tol > 0.0 && pb.floor_stop, bad = false;
  for (int n = 0; n < pb.N; ++n) {
    const double r = res[n];
    sc->residual[n] = r;
    pb.hist[(int64_t)sc->k * pb.N + n] = r;
    if (!(r < pb.tol)) conv = false;
    if (!(r < floor_lvl)) at_floor = false;
    if (!isfinite(r)) bad = true;
  }
  if (!isfinite(dmax)) bad = true;
  sc->mu = fmin(pb.rho * sc->mu, pb.mu_max);
  sc->k += 1;
  if (bad) {
    sc->done = 3;
  } else if (conv) {
    sc->converged = 1;
    sc->done = 1;
  } else if (at_floor) {
    sc->done = 4;
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
  for (int e = threadIdx.x; e < g.I * g.T * kRT; e += blockDim.x) {
    // Us tile-major: tile t, row i, column kRT t + cc
    const int t = e / (g.I * kRT), rem = e - t * g.I * kRT;
    const int i = rem / kRT, c = t * kRT + rem % kRT;
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
    for (int e = threadIdx.x; e < (kMaxN + 1) * kResSlots; e += blockDim.x)
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
      for (int n = 0; n < pb.N; ++n) acc += pb.alpha[n] * recon1(pb, n, x);
      X[x] = (S)(acc / wsum);
    }
    if (E) E[x] = pb.T[x] - pb.D[x];
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_component(Problem<S> pb, int n, S* Z) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < pb.numel;
       x += (int64_t)gridDim.x * blockDim.x) {
    Z[x] = (S)recon1(pb, n, x);
  }
}

static int elem_grid(int64_t work) {
  int64_t b = (work + 255) / 256;
  if (b > 256 * 16) b = 256 * 16;
  if (b < 1) b = 1;
  return (int)b;
}

int fused_blocks(int64_t numel, int vec) { return elem_grid(numel / vec); }

// The fused pass folds in the GEMM-M of modes 0 and 1 (order 4, ranks within
// one tile, 32-bit offsets) when the mode-1 slab, S = B_1 / vec chunks with one
// index i_1, holds at least four block sweeps of 256 chunks: blocks of mcb
// chunks, mcb the smallest divisor of S not below max(1024, nchunk / 4096), so
// that every block lies inside one slab of both merged modes and the grid
// stays near the 4096 blocks of the plain pass.  Measured (per iteration,
// merged against separate GEMM-M): 64^4 FP64 R_n = 6 0.707 against 0.837 ms,
// R_n = 16 1.218 against 1.242; FP32 R_n = 6, 8, 10 0.368 / 0.402 / 0.445
// against 0.413 / 0.436 / 0.474 ms, but R_n = 12 0.611 against 0.503 (the
// kept P_n columns and sums take the FP32 pass to one wave per SIMD), so FP32
// states merge up to rank 10.  Blocks of fewer sweeps spend too much on their
// set-up and the partial sums: 32 x 48 x 40 x 56 (S = 560 FP32 chunks, one
// sweep) ran the pass at 79 against 40 us.  Folding in one mode of a 3-way
// tensor, 200^3 FP32 or the video-shaped workload, costs the pass more than it
// saves, since the kept P_n columns and sums halve its occupancy.
void merge_plan(const int64_t* dims, int N, int64_t numel, int vec, int max_rank, int state_bytes,
                bool idx32, int* mmerge, int64_t* mcb, int* blocks, int* mfull) {
  *mmerge = 0;
  *mcb = 0;
  *mfull = 0;
  *blocks = fused_blocks(numel, vec);
  if (!idx32 || max_rank > kRT || N != 4) return;
  if (state_bytes == 4 && max_rank > 10) return;
  const int64_t nchunk = numel / vec;
  for (int d = 1; d >= 1; --d) {
    int64_t B = 1;
    for (int m = d + 1; m < N; ++m) B *= dims[m];
    if (B % vec) continue;
    const int64_t S = B / vec;
    if (S < 1024) continue;
    int64_t cb = std::max<int64_t>(1024, (nchunk + 4095) / 4096);
    if (cb >= S) cb = S;
    while (S % cb) ++cb;
    const int64_t nb = nchunk / cb;
    if (nb > 65535) return;
    *mmerge = d + 1;
    *mcb = cb;
    *blocks = (int)nb;
    // the fast modes too (FP64, ranks up to 6, the 16-byte vector path) when
    // every chunk of a thread has the same last-mode columns (Q | 256 and Q |
    // mcb), a row group lies in one wave (Q <= 64) and the block's rows fit
    // the LDS stage
    const int64_t Q = dims[N - 1] / vec;
    *mfull = state_bytes == 8 && vec == 2 && max_rank <= 6 && Q <= 64 && 256 % Q == 0 &&
             cb % Q == 0 &&
             cb / Q <= kStageRows;
    return;
  }
}

template <typename S, int NN, int RP, int MM>
static void fused_idx(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int grid = make_batch(ls, b, [](const Problem<S>& p) { return p.fused_blocks; });
  if constexpr (MM > 0) {
    // merged problems (32-bit offsets by construction)
    hipLaunchKernelGGL((k_fused<S, NN, RP, uint32_t, false, MM>), dim3(grid), dim3(256), 0, s, b);
  } else {
    bool idx32 = true;
    for (int r = 0; r < ls.count; ++r) idx32 = idx32 && ls.host[r]->idx32;
    // the mode-1 order over the XCDs (Problem::fsplit1) for a launch of one
    // problem whose blocks fill whole XCD rounds; the traversal order changes
    // no result
    const bool split1 = idx32 && ls.count == 1 && ls.host[0]->fsplit1 && grid % kXcds == 0;
    if (split1)
      hipLaunchKernelGGL((k_fused<S, NN, RP, uint32_t, true, 0>), dim3(grid), dim3(256), 0, s, b);
    else if (idx32)
      hipLaunchKernelGGL((k_fused<S, NN, RP, uint32_t, false, 0>), dim3(grid), dim3(256), 0, s, b);
    else  // offsets beyond 32 bits: 64-bit indexing, full rank tile (or the tile loop)
      hipLaunchKernelGGL((k_fused<S, NN, RP == 0 ? 0 : kRT, uint64_t, false, 0>), dim3(grid),
                         dim3(256), 0, s, b);
  }
}

template <typename S, int NN, int RP, int MM>
static void mrefresh_idx(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int grid = make_batch(ls, b, [](const Problem<S>& p) { return p.fused_blocks; });
  hipLaunchKernelGGL((k_mrefresh<S, NN, RP, MM>), dim3(grid), dim3(256), 0, s, b);
}

// The rank loop is unrolled to the largest R_n of the set, rounded up to even
// for orders up to 4 and to a multiple of 4 above.  REFRESH: the merged
// modes' GEMM-M partials only (k_mrefresh).
template <typename S, int NN, int MM, bool REFRESH = false>
static void fused_n(const LaunchSet<S>& ls, hipStream_t s) {
  int rmax = 1;
  for (int r = 0; r < ls.count; ++r)
    for (int n = 0; n < ls.host[r]->N; ++n) rmax = std::max(rmax, ls.host[r]->g[n].R);
  auto go = [&](auto rp) {
    constexpr int RP = decltype(rp)::value;
    if constexpr (REFRESH)
      mrefresh_idx<S, NN, RP, MM>(ls, s);
    else
      fused_idx<S, NN, RP, MM>(ls, s);
  };
  if constexpr (NN <= 4) {
    // orders up to 4: the rank loop is unrolled to R rounded up to even (the
    // pass is bound by its load instructions, one per rank and mode)
    switch ((rmax + 1) / 2) {
      case 1: go(std::integral_constant<int, 2>{}); return;
      case 2: go(std::integral_constant<int, 4>{}); return;
      case 3: go(std::integral_constant<int, 6>{}); return;
      case 4: go(std::integral_constant<int, 8>{}); return;
      case 5: go(std::integral_constant<int, 10>{}); return;
      case 6: go(std::integral_constant<int, 12>{}); return;
      case 7: go(std::integral_constant<int, 14>{}); return;
      default: go(std::integral_constant<int, 16>{}); return;
    }
  } else {
    if (rmax <= 4)
      go(std::integral_constant<int, 4>{});
    else if (rmax <= 8)
      go(std::integral_constant<int, 8>{});
    else if (rmax <= 12)
      go(std::integral_constant<int, 12>{});
    else
      go(std::integral_constant<int, 16>{});
  }
}

// fused_n per rank class: a problem's reconstruction loads scale with the
// unrolled rank bound RP, so the problems of a set go out in one launch per
// class of their own largest rank (a rank-3 solve in a batch with a rank-15
// one would otherwise run the rank-16 loop).  The padded rank terms are exact
// zeros, so a problem's results do not depend on the class it launches with.
template <typename S, int NN, int MM, bool REFRESH = false>
static void fused_by_rank(const LaunchSet<S>& ls, hipStream_t s) {
  constexpr int kClasses = 8;
  LaunchSet<S> cls[kClasses];
  for (int r = 0; r < ls.count; ++r) {
    int rm = 1;
    for (int n = 0; n < ls.host[r]->N; ++n) rm = std::max(rm, ls.host[r]->g[n].R);
    const int c = NN <= 4 ? std::min(kClasses - 1, (rm - 1) / 2) : std::min(3, (rm - 1) / 4);
    LaunchSet<S>& d = cls[c];
    d.host[d.count] = ls.host[r];
    d.dev[d.count] = ls.dev[r];
    ++d.count;
  }
  for (int c = 0; c < kClasses; ++c)
    if (cls[c].count) fused_n<S, NN, MM, REFRESH>(cls[c], s);
}

// Problems of a set by their number of merged modes (0, 1 or 2; 3: every
// mode, Problem::mfull).  The fast modes' code is compiled for ranks up to 6
// only, so those problems go out in launches of their own, whose rank bound
// is theirs.
template <typename S>
static void split_merged(const LaunchSet<S>& ls, LaunchSet<S> (&out)[4]) {
  for (int m = 0; m < 4; ++m) out[m].count = 0;
  for (int r = 0; r < ls.count; ++r) {
    LaunchSet<S>& d = out[ls.host[r]->mfull ? 3 : ls.host[r]->mmerge];
    d.host[d.count] = ls.host[r];
    d.dev[d.count] = ls.dev[r];
    ++d.count;
  }
}

// All problems of a set have the same order N (the batch driver groups them).
// Problems with some R_n > kRT take the tile-looped rank path (RP = 0);
// problems with merged modes (order 4 only) their own instantiations.
template <typename S>
void launch_fused(const LaunchSet<S>& ls, hipStream_t s) {
  LaunchSet<S> nar, wid;
  split_wide(ls, nar, wid);
  if (nar.count) {
    LaunchSet<S> mg[4];
    split_merged(nar, mg);
    const int N = nar.host[0]->N;
    if (mg[0].count) {
      switch (N) {
        case 2: fused_by_rank<S, 2, 0>(mg[0], s); break;
        case 3: fused_by_rank<S, 3, 0>(mg[0], s); break;
        case 4: fused_by_rank<S, 4, 0>(mg[0], s); break;
        case 5: fused_by_rank<S, 5, 0>(mg[0], s); break;
        case 6: fused_by_rank<S, 6, 0>(mg[0], s); break;
        case 7: fused_by_rank<S, 7, 0>(mg[0], s); break;
        default: fused_by_rank<S, 8, 0>(mg[0], s); break;
      }
    }
    if (mg[2].count) fused_by_rank<S, 4, 2>(mg[2], s);
    if (mg[3].count) fused_by_rank<S, 4, 2>(mg[3], s);
  }
  if (wid.count) {
    switch (wid.host[0]->N) {
      case 2: fused_idx<S, 2, 0, 0>(wid, s); break;
      case 3: fused_idx<S, 3, 0, 0>(wid, s); break;
      case 4: fused_idx<S, 4, 0, 0>(wid, s); break;
      case 5: fused_idx<S, 5, 0, 0>(wid, s); break;
      case 6: fused_idx<S, 6, 0, 0>(wid, s); break;
      case 7: fused_idx<S, 7, 0, 0>(wid, s); break;
      default: fused_idx<S, 8, 0, 0>(wid, s); break;
    }
  }
}

template <typename S>
void launch_mrefresh(const LaunchSet<S>& ls, hipStream_t s) {
  LaunchSet<S> mg[4];
  split_merged(ls, mg);
  if (mg[2].count) fused_by_rank<S, 4, 2, true>(mg[2], s);
  if (mg[3].count) fused_by_rank<S, 4, 2, true>(mg[3], s);
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
  template void launch_component<S>(const Problem<S>&, int, S*, hipStream_t); \
  template void launch_mrefresh<S>(const LaunchSet<S>&, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace pasd
