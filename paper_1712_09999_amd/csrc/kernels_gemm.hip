// Unfolding GEMMs of the PASD iteration on gfx950 matrix cores.
//
//   GEMM-M : M_n = G_n P_n^T      (I_n x R_n, contraction over the J_n columns)
//            whose orthonormal basis is the new active subspace U_n
//            (Procrustes step, eqs. (9)-(10));
//   GEMM-P : P_n = U_n^T G_n      (R_n x J_n, contraction over I_n),
//            the matrix whose SVT is V_n (eq. (13));
//   Gram   : S_n = P_n P_n^T      (R_n x R_n, FP64), for the SVT by eigensolver;
//
// with G_n = T_(n) - E_(n) + Y_n,(n) / mu formed on the fly from D = T - E and
// Y_n (definition under eq. (9)); G is never stored.
//
// All three use v_mfma_{f32,f64}_16x16x4 with the rank padded to one 16-wide
// tile (ranks above 16 run as several one-tile problems, see for_tile_sets,
// and the Gram has a rank-wide variant, k_gram_w).  The unfolding is read in place through its (A, I, B) geometry.  The
// contraction index inside one MFMA is permuted freely (both operands use the
// same permutation), which lets every lane issue 4-element vector loads along
// the contiguous direction of the tensor.  Split-K partial sums are reduced
// in LDS within a block and across blocks by a separate, fixed-order pass, so
// results are bitwise reproducible.
#include <algorithm>
#include <type_traits>

#include "pasd_internal.hpp"

namespace pasd {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

// Loads of the streaming loops go through explicitly global pointers: generic
// "flat" loads also occupy the LDS wait counter, so every wait for them would
// drain LDS traffic too.
#define PASD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gld(const void* p) {
  return *(const PASD_GLOBAL T*)p;
}

template <typename S> struct MM;
// Operand layout of both 16x16x4 instructions: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16].  Result element v of lane l is D[row(l / 16, v)][l % 16]
// with row = 4 (l/16) + v for the f32 instruction and 4 v + l/16 for the f64
// one (measured on gfx950).
template <> struct MM<float> {
  typedef f4v acc_t;
  typedef f4v vec_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};
template <> struct MM<double> {
  typedef d4v acc_t;
  typedef d4v vec_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return 4 * v + q; }
};

__device__ __forceinline__ d4v mma64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Split-BF16 products on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16).
// Every FP32 operand x is written as x = h1 + h2 + h3 + e with h1 = bf16(x),
// h2 = bf16(x - h1), h3 = bf16(x - h1 - h2), each BF16 rounding to nearest
// even; both differences are exact in FP32 and |e| <= 2^-25 |x|.  The product
// a b is taken as the six terms a1 b1 + a2 b1 + a1 b2 + a2 b2 + a1 b3 + a3 b1
// (the dropped terms are below 2^-23 |a b|), each exact in FP32 and summed
// with FP32 accumulation, so the GEMM keeps FP32 accuracy while every
// multiplication runs on the BF16 matrix cores.
//
// The BF16 instruction takes 8 BF16 values of A and of B per lane where the
// FP32 one takes one each: lane l supplies A[l % 16][k] and B[k][l % 16] for
// the same eight contraction indices k, and the result layout is the f32
// instruction's (row 4 (l/16) + v, column l % 16; checked on gfx950 with an
// in-bounds probe).  One FP32 MFMA term A[m][k] B[k][n] becomes one BF16 MFMA
// whose eight slots hold the six split products of that term (two slots zero);
// the contraction index is still the lane group l / 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);  // inf / NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

struct Split3 {
  uint32_t h1, h2, h3;  // BF16 bit patterns in the low 16 bits
};

__device__ __forceinline__ Split3 split3(float x) {
  Split3 s;
  s.h1 = bf16_rne_bits(x);
  const float r1 = x - __uint_as_float(s.h1 << 16);
  s.h2 = bf16_rne_bits(r1);
  const float r2 = r1 - __uint_as_float(s.h2 << 16);
  s.h3 = bf16_rne_bits(r2);
  return s;
}

__device__ __forceinline__ f4v mma_split_bf16(float a, float b, f4v acc) {
  const Split3 x = split3(a), y = split3(b);
  // slots:  A = a1 a2 | a1 a2 | a1 a3 | 0 0,  B = b1 b1 | b2 b2 | b3 b1 | 0 0
  const u4v va = u4v{x.h1 | (x.h2 << 16), x.h1 | (x.h2 << 16), x.h1 | (x.h3 << 16), 0u};
  const u4v vb = u4v{y.h1 | (y.h1 << 16), y.h2 | (y.h2 << 16), y.h3 | (y.h1 << 16), 0u};
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, va),
                                                 __builtin_bit_cast(bf16x8, vb), acc, 0, 0, 0);
}

// One MFMA term A[m][k] B[k][n] += a b: FP32 / FP64 matrix cores, or with BF
// the split-BF16 form above (FP32 state only).
template <bool BF, typename S>
__device__ __forceinline__ typename MM<S>::acc_t mma_op(S a, S b, typename MM<S>::acc_t acc) {
  if constexpr (BF) {
    static_assert(sizeof(S) == 4, "split-BF16 operands come from the FP32 state");
    return mma_split_bf16(a, b, acc);
  } else {
    return MM<S>::mma(a, b, acc);
  }
}

// Four values of G = D + Y * inv_mu at element offsets off[t] (t < nvalid).
// `contig` means the four offsets are consecutive and 4-aligned.
template <typename S>
__device__ __forceinline__ void load_g4(const S* __restrict__ D, const S* __restrict__ Y,
                                        const int64_t off[4], bool contig, int nvalid, S inv_mu,
                                        S g[4]) {
  typedef typename MM<S>::vec_t V;
  if (contig && nvalid == 4) {
    V d = *reinterpret_cast<const V*>(D + off[0]);
    V y = *reinterpret_cast<const V*>(Y + off[0]);
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = d[t] + y[t] * inv_mu;
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = (t < nvalid) ? D[off[t]] + Y[off[t]] * inv_mu : S(0);
  }
}

// ---------------------------------------------------------------------------
// GEMM-P.  Column scheme (B > 1): one block = 64 unfolding columns, its 4 waves
// split the I_n contraction; lane (p, q) holds columns j0 + 4p .. +3 of row
// i0 + q.  MFMA t: A[r][k] = U[i0+k][r], B[k][c] = G[i0+k][j0 + 4c + t].
// When 256 divides B_n, a block takes 256 columns instead, wave w the 64
// from j0 + 64 w, each wave the whole contraction (no sum across waves): every
// row is then read in 2 KB (FP64) runs rather than 512-byte ones (64^4,
// modes 0 and 1: 119.6 -> 110.5 us FP64, FP32 and split-BF16 9 and 13 us less).
// Row scheme (B == 1, the last mode): one wave = 16 rows a, lane (p, q) reads
// G[a0+p][i0+4q .. +3]; A[a][k] = G, B[k][r] = U, all four t accumulate into
// one tile since they share the output.
// ---------------------------------------------------------------------------

// Orders the LDS accesses of one wave: the compiler keeps them on their side
// of this point, and the LDS executes a wave's accesses in issue order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// GEMM-P of the last two modes together (Problem::gp2: I_{N-2} = I_{N-1} =
// 64).  The 64 x 64 slab of index a over modes 0 .. N-3 holds tile a of both
// unfoldings: columns 64 a .. 64 a + 63 of mode N-2 (contraction over
// i_{N-2}) and rows 64 a .. 64 a + 63 of mode N-1 (contraction over
// i_{N-1}).  One block reads D there once for both modes, and Y_{N-2},
// Y_{N-1} once each, instead of D twice.  Wave w takes rows i_{N-2} = 16 w ..
// 16 w + 15: for mode N-2 the column scheme's fragments (lane (p, q): rows
// 16 w + 4 k + q, columns 4 p .. 4 p + 3) and its LDS sum over the waves, for
// mode N-1 the row scheme's (row 16 w + p, columns 16 k + 4 q .. + 3), with D
// brought into them by a transpose through the wave's own LDS region.  Both
// modes' products and sums run in the one-mode kernel's order, so P_n is
// bitwise the same as there.
// (At most 168 registers, three waves per SIMD: FP64 fits without spilling,
// 208 -> 202 us for the GEMM-P of 64^4 against two waves.)
template <typename S, bool BF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_gemm_p2(Batch<S> bt) {
  typedef typename MM<S>::acc_t Acc;
  typedef typename MM<S>::vec_t V;
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int64_t a = blockIdx.x - bt.start[req];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  const int n2 = pb.N - 2, n3 = pb.N - 1;
  const ModeGeom g2 = pb.g[n2], g3 = pb.g[n3];
  const ModeBufs<S> m2 = pb.m[n2], m3 = pb.m[n3];
  const S inv_mu = S(1.0 / pb.sc->mu);
  // per wave 1024 elements: first the transposed 16 x 64 rows of D (4-element
  // groups of row r at group index g ^ (r & 15)), then the wave's sums
  __shared__ __align__(32) S red[4][64][16];
  S* buf = &red[wave][0][0];
  const int64_t base = a * 4096;
  V d[4], y2[4], y3[4];
  S u2[4], u3[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int row = 16 * wave + 4 * k + q;
    d[k] = *reinterpret_cast<const V*>(pb.D + base + row * 64 + 4 * p);
    y2[k] = *reinterpret_cast<const V*>(m2.Y + base + row * 64 + 4 * p);
    u2[k] = m2.Us[row * kRT + p];
    y3[k] = *reinterpret_cast<const V*>(m3.Y + base + (16 * wave + p) * 64 + 16 * k + 4 * q);
#pragma unroll
    for (int t = 0; t < 4; ++t) u3[k][t] = m3.Us[(16 * k + 4 * q + t) * kRT + p];
  }
  __builtin_amdgcn_sched_barrier(0);
  Acc acc2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc2[t] = Acc{0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc2[t] = mma_op<BF, S>(u2[k], d[k][t] + y2[k][t] * inv_mu, acc2[t]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = 4 * k + q;
    *reinterpret_cast<V*>(buf + r * 64 + 4 * (p ^ r)) = d[k];
  }
  wave_lds_sync();
  Acc acc3 = Acc{0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const V d3 = *reinterpret_cast<const V*>(buf + p * 64 + 4 * ((4 * k + q) ^ p));
#pragma unroll
    for (int t = 0; t < 4; ++t) acc3 = mma_op<BF, S>(d3[t] + y3[k][t] * inv_mu, u3[k][t], acc3);
  }
  // acc3[v] = P_{N-1}[p][64 a + 16 w + row(q, v)]
  if (p < g3.R) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      m3.P[(int64_t)p * g3.J + a * 64 + 16 * wave + MM<S>::row(q, v)] = acc3[v];
  }
  wave_lds_sync();  // the transposed rows are read out before the sums overwrite them
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][lane][t * 4 + v] = acc2[t][v];
  __syncthreads();
  if (wave == 0) {
    // P_{N-2}[r][64 a + 4 p + t], r = row(q, v), in the column scheme's order
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = MM<S>::row(q, v);
      if (r >= g2.R) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        S s = red[0][lane][t * 4 + v] + red[1][lane][t * 4 + v] + red[2][lane][t * 4 + v] +
              red[3][lane][t * 4 + v];
        m2.P[(int64_t)r * g2.J + a * 64 + 4 * p + t] = s;
      }
    }
  }
}

template <typename S, bool BF>
__global__ void __launch_bounds__(256) k_gemm_p(Batch<S> bt) {
  typedef typename MM<S>::acc_t Acc;
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_GEMM_P], pb.N, lb);
  int64_t tile = lb - pb.kb[KB_GEMM_P][n];
  {
    // Blocks are dealt to the 8 XCDs in turn; give each XCD a contiguous run
    // of tiles, so that the cache lines two neighbouring tiles share (rows
    // shorter than a tile's span) are fetched into one L2.
    const int nt = pb.kb[KB_GEMM_P][n + 1] - pb.kb[KB_GEMM_P][n];
    tile = xcd_order((int)tile, nt, bt.start[req] + pb.kb[KB_GEMM_P][n]);
  }
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const S inv_mu = S(1.0 / pb.sc->mu);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  const S* __restrict__ Us = mb.Us;

  if (g.B > 1) {
    __shared__ S red[4][64][16];
    // B_n a multiple of 256 (every 256-column tile full, inside one row run):
    // wave w takes columns 64 w .. 64 w + 63 of the tile over the whole contraction
    const bool side = (g.B % 256) == 0;
    const int64_t j4 = side ? tile * 256 + wave * 64 + 4 * p : tile * 64 + 4 * p;
    int64_t off[4];
    int nvalid = 0;
    const bool contig = (g.B % 4) == 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t j = j4 + t;
      const int64_t jj = j < g.J ? j : 0;
      const int64_t a = jj / g.B, b = jj - a * g.B;
      off[t] = a * (int64_t)g.I * g.B + b;
      nvalid += (j < g.J) ? 1 : 0;
    }
    const int rows_per_wave = ((g.I + 15) / 16) * 4;
    const int kbeg = side ? 0 : wave * rows_per_wave;
    const int kend = side ? g.I : min(g.I, kbeg + rows_per_wave);
    Acc acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = Acc{0, 0, 0, 0};
    typedef typename MM<S>::vec_t V;
    if (contig && (side || (tile + 1) * 64 <= g.J)) {
      // all 64 columns valid: unconditional vector loads (rows past kend are
      // clamped to a valid row and masked), so unrolled iterations overlap
      const S* __restrict__ Db = pb.D + off[0];
      const S* __restrict__ Yb = mb.Y + off[0];
      // four K-steps (16 rows) per pass, all loads issued before the MFMAs;
      // a masked row contributes u = 0 times a finite value of a valid row
      for (int i0 = kbeg; i0 < kend; i0 += 16) {
        V d[4], y[4];
        S u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const bool ok = i0 + 4 * k + q < kend;
          const int i = ok ? i0 + 4 * k + q : kbeg;
          d[k] = *reinterpret_cast<const V*>(Db + (int64_t)i * g.B);
          y[k] = *reinterpret_cast<const V*>(Yb + (int64_t)i * g.B);
          const S uu = Us[(int64_t)i * kRT + p];
          u[k] = ok ? uu : S(0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[t] = mma_op<BF, S>((u[k]), (d[k][t] + y[k][t] * inv_mu), acc[t]);
      }
    } else {
      for (int i0 = kbeg; i0 < kend; i0 += 4) {
        const int i = i0 + q;
        S gv[4] = {0, 0, 0, 0};
        S u = 0;
        if (i < kend) {
          int64_t o[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) o[t] = off[t] + (int64_t)i * g.B;
          load_g4<S>(pb.D, mb.Y, o, contig, nvalid, inv_mu, gv);
          u = Us[(int64_t)i * kRT + p];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mma_op<BF, S>((u), (gv[t]), acc[t]);
      }
    }
    if (side) {
      // the wave's own 64 columns are complete: no sum across waves
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = MM<S>::row(q, v);
        if (r >= g.R) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) mb.P[(int64_t)r * g.J + j4 + t] = acc[t][v];
      }
      return;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wave][lane][t * 4 + v] = acc[t][v];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = MM<S>::row(q, v);
        if (r >= g.R) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (t >= nvalid) continue;
          S s = red[0][lane][t * 4 + v] + red[1][lane][t * 4 + v] + red[2][lane][t * 4 + v] +
                red[3][lane][t * 4 + v];
          mb.P[(int64_t)r * g.J + j4 + t] = s;
        }
      }
    }
  } else {
    // Row scheme: rows a = tile*64 + wave*16 + p.
    const int64_t a0 = tile * 64 + wave * 16;
    const int64_t arow = a0 + p;
    const bool rowok = arow < g.A;
    const bool contig = (g.I % 4) == 0;
    Acc acc = Acc{0, 0, 0, 0};
    if (contig) {
      // unconditional vector loads: the row is clamped to a valid one and
      // masked; chunks past I are clamped to the last chunk and masked
      typedef typename MM<S>::vec_t V;
      const int64_t ar = rowok ? arow : g.A - 1;
      const S* __restrict__ Db = pb.D + ar * g.I;
      const S* __restrict__ Yb = mb.Y + ar * g.I;
      // four 16-wide chunks per pass, all loads issued before the MFMAs.
      // Lane (p, q) supplies A[p][q] (row a0 + p) and B[q][p] (column chunk
      // q, rank p): a chunk past I is masked in B, a row past A in A.
      for (int i0 = 0; i0 < g.I; i0 += 64) {
        V d[4], y[4];
        S u[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int iq = i0 + 16 * k + 4 * q;
          const bool ok = iq < g.I;
          const int i = ok ? iq : g.I - 4;
          d[k] = *reinterpret_cast<const V*>(Db + i);
          y[k] = *reinterpret_cast<const V*>(Yb + i);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const S uu = Us[(int64_t)(i + t) * kRT + p];
            u[k][t] = ok ? uu : S(0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc = mma_op<BF, S>((rowok ? d[k][t] + y[k][t] * inv_mu : S(0)), (u[k][t]), acc);
      }
    } else {
      for (int i0 = 0; i0 < g.I; i0 += 16) {
        const int i = i0 + 4 * q;
        const int nv = max(0, min(4, g.I - i));
        S gv[4] = {0, 0, 0, 0};
        if (rowok && nv > 0) {
          int64_t o[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) o[t] = arow * g.I + i + t;
          load_g4<S>(pb.D, mb.Y, o, contig, nv, inv_mu, gv);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const S u = (t < nv) ? Us[(int64_t)(i + t) * kRT + p] : S(0);
          acc = mma_op<BF, S>((gv[t]), (u), acc);
        }
      }
    }
    // D[m][n = p] = P[r = p][a0 + m], m = row(q, v)
    if (p < g.R) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t a = a0 + MM<S>::row(q, v);
        if (a < g.A) mb.P[(int64_t)p * g.J + a] = acc[v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// GEMM-M split-K partials.  Block = 8 waves; the block owns a contiguous
// range of the contraction (columns j for B > 1, rows a for B == 1) and
// writes one partial M[I][16] (FP64) after reducing its waves in LDS.
// Column scheme: K-step = 16 columns, lane (p, q) holds columns j0+4q..+3;
// for row block ib: A[i][k] = G[16ib + i][col], B[k][r] = P[r][col].
// Row scheme: K-step = 4 rows a (k = q); lane (p, q) holds G[a0+q][64c+4p..+3];
// MFMA (c, t): A[m][k] = G[a0+k][64c + 4m + t], B[k][r] = P[r][a0+k].
// ---------------------------------------------------------------------------

constexpr int kMWaves = 8;

template <typename S, bool BF, bool RS, bool NARROW>
__global__ void __launch_bounds__(512) k_gemm_m(Batch<S> bt) {
  typedef typename MM<S>::acc_t Acc;
  typedef typename MM<S>::vec_t V;
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_GEMM_M], pb.N, lb);
  const int blk = lb - pb.kb[KB_GEMM_M][n];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const S inv_mu = S(1.0 / pb.sc->mu);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  __shared__ double red[kMWaves][64][4];
  double* __restrict__ out = mb.Mpart + (int64_t)blk * g.I * g.R;  // [I][R] partial

  const int64_t csteps = (g.J + 15) / 16;
  const int64_t cper = (csteps + mb.mblocks - 1) / mb.mblocks;
  // RS (the instantiation for a launch of one problem): with fewer than 12 row
  // blocks most waves would own no rows and with fewer than 8 steps per block
  // the split over steps below needs fewer round trips, so those take it; a
  // batch of many problems (serving) uses the other instantiation, where the
  // split over steps measured faster.
  if (RS && g.B > 1 && (g.B % 4) == 0 && (g.J % 4) == 0 && cper >= 8 && g.I > 11 * 16 &&
      min(csteps, (int64_t)(blk + 1) * cper) <= g.J / 16) {
    // Column scheme, rows split over the waves: every 16-column step of the
    // block is full and 4-aligned.  Wave w owns row blocks rb0, rb0 + 1 (16
    // rows each; passes of 16 row blocks) and runs through all of the block's
    // steps, 4 at a time, so each lane reads 64 contiguous bytes of its row per
    // tensor and every row is read in 256-byte runs; no cross-wave reduction.
    constexpr int RBW = 2, KS = 4;
    const int64_t sbeg = (int64_t)blk * cper;
    const int64_t send = min(csteps, sbeg + cper);
    const int nib = (g.I + 15) / 16;
    const bool j32 = g.J < (int64_t(1) << 31);
    const FastDiv fdb = pb.fd_b[n];
    const int pr = min(p, g.R - 1);  // lanes p >= R read row R-1 (cached) and mask it
    for (int rg = 0; rg < nib; rg += RBW * kMWaves) {
      const int rb0 = rg + RBW * wave;
      Acc acc[RBW];
#pragma unroll
      for (int u = 0; u < RBW; ++u) acc[u] = Acc{0, 0, 0, 0};
      auto step = [&](int64_t st0, auto kcount) {
        constexpr int K = decltype(kcount)::value;
        V pv[K], dv[RBW][K], yv[RBW][K];
#pragma unroll
        for (int ks = 0; ks < K; ++ks) {
          const int64_t j4 = (st0 + ks) * 16 + 4 * q;
          const int64_t a = j32 ? (int64_t)fastdiv((uint32_t)j4, fdb) : j4 / g.B;
          const int64_t b = j4 - a * g.B;
          const S* dp = pb.D + a * (int64_t)g.I * g.B + b;
          const S* yp = mb.Y + a * (int64_t)g.I * g.B + b;
          pv[ks] = gld<V>(mb.P + (int64_t)pr * g.J + j4);
#pragma unroll
          for (int u = 0; u < RBW; ++u) {
            const int64_t i = min((rb0 + u) * 16 + p, g.I - 1);
            dv[u][ks] = gld<V>(dp + i * g.B);
            yv[u][ks] = gld<V>(yp + i * g.B);
          }
        }
        // every load of the steps is in flight before the first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < K; ++ks) {
          const V pvv = p < g.R ? pv[ks] : V{0, 0, 0, 0};
#pragma unroll
          for (int u = 0; u < RBW; ++u) {
            const bool ok = (rb0 + u) * 16 + p < g.I;
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[u] = mma_op<BF, S>((ok ? dv[u][ks][t] + yv[u][ks][t] * inv_mu : S(0)),
                                  (pvv[t]), acc[u]);
          }
        }
      };
      int64_t st = sbeg;
      for (; st + KS <= send; st += KS) step(st, std::integral_constant<int, KS>{});
      for (; st < send; ++st) step(st, std::integral_constant<int, 1>{});
#pragma unroll
      for (int u = 0; u < RBW; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = (rb0 + u) * 16 + MM<S>::row(q, v);
          if (i < g.I && p < g.R) out[(int64_t)i * g.R + p] = (double)acc[u][v];
        }
    }
  } else if (g.B > 1) {
    // row blocks per pass (register budget); NARROW launches (every I_n <= 64)
    // need at most 4
    constexpr int IBP = (sizeof(S) == 4 && !NARROW) ? 8 : 4;
    const int64_t nsteps = (g.J + 15) / 16;
    const int64_t per_blk = (nsteps + mb.mblocks - 1) / mb.mblocks;
    const int64_t sbeg = (int64_t)blk * per_blk;
    const int64_t send = min(nsteps, sbeg + per_blk);
    const bool contig = (g.B % 4) == 0;
    const bool pvec = (g.J % 4) == 0;
    const int nib = (g.I + 15) / 16;
    const int pr = min(p, g.R - 1);  // lanes p >= R read row R-1 (cached) and mask it
    for (int ib0 = 0; ib0 < nib; ib0 += IBP) {
      Acc acc[IBP];
#pragma unroll
      for (int u = 0; u < IBP; ++u) acc[u] = Acc{0, 0, 0, 0};
      // steps whose 16 columns are all valid, on 4-aligned contiguous columns:
      // unconditional vector loads (rows past I and P_n rows past R clamped
      // and masked), so that the loads of all row blocks overlap
      const int64_t full_end = (contig && pvec) ? min(send, g.J / 16) : sbeg;
      const bool j32 = g.J < (int64_t(1) << 31);
      const FastDiv fdb = pb.fd_b[n];
      int64_t st = sbeg + wave;
      for (; st < full_end; st += kMWaves) {
        const int64_t j4 = st * 16 + 4 * q;
        const int64_t a = j32 ? (int64_t)fastdiv((uint32_t)j4, fdb) : j4 / g.B;
        const int64_t b = j4 - a * g.B;
        const S* dp = pb.D + a * (int64_t)g.I * g.B + b;
        const S* yp = mb.Y + a * (int64_t)g.I * g.B + b;
        const V pv0 = gld<V>(mb.P + (int64_t)pr * g.J + j4);
        V dv[IBP], yv[IBP];
#pragma unroll
        for (int u = 0; u < IBP; ++u) {
          const int64_t i = min((ib0 + u) * 16 + p, g.I - 1);
          dv[u] = gld<V>(dp + i * g.B);
          yv[u] = gld<V>(yp + i * g.B);
        }
        // every load of the step is in flight before the first use
        __builtin_amdgcn_sched_barrier(0);
        const V pvv = p < g.R ? pv0 : V{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < IBP; ++u) {
          // row blocks past I (the last pass) compute on zeros, no branch
          const bool ok = (ib0 + u) * 16 + p < g.I;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[u] = mma_op<BF, S>((ok ? dv[u][t] + yv[u][t] * inv_mu : S(0)), (pvv[t]), acc[u]);
        }
      }
      for (; st < send; st += kMWaves) {
        const int64_t j4 = st * 16 + 4 * q;
        int64_t off[4];
        int nvalid = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int64_t j = j4 + t;
          const int64_t jj = j < g.J ? j : 0;
          const int64_t a = jj / g.B, b = jj - a * g.B;
          off[t] = a * (int64_t)g.I * g.B + b;
          nvalid += (j < g.J) ? 1 : 0;
        }
        S pv[4] = {0, 0, 0, 0};
        if (p < g.R) {
          const S* prow = mb.P + (int64_t)p * g.J;
          if (pvec && nvalid == 4) {
            V v = *reinterpret_cast<const V*>(prow + j4);
#pragma unroll
            for (int t = 0; t < 4; ++t) pv[t] = v[t];
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) pv[t] = (t < nvalid) ? prow[j4 + t] : S(0);
          }
        }
#pragma unroll
        for (int u = 0; u < IBP; ++u) {
          const int i = (ib0 + u) * 16 + p;
          if (ib0 + u >= nib) break;
          S gv[4] = {0, 0, 0, 0};
          if (i < g.I && nvalid > 0) {
            int64_t o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) o[t] = off[t] + (int64_t)i * g.B;
            load_g4<S>(pb.D, mb.Y, o, contig, nvalid, inv_mu, gv);
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[u] = mma_op<BF, S>((gv[t]), (pv[t]), acc[u]);
        }
      }
      // reduce the waves and write rows i = 16(ib0+u) + 4q + v, column r = p
      for (int u = 0; u < IBP; ++u) {
        if (ib0 + u >= nib) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave][lane][v] = (double)acc[u][v];
        __syncthreads();
        if (threadIdx.x < 256) {
          const int l = threadIdx.x >> 2, v = threadIdx.x & 3;
          double s = 0;
#pragma unroll
          for (int w = 0; w < kMWaves; ++w) s += red[w][l][v];
          const int i = (ib0 + u) * 16 + MM<S>::row(l >> 4, v);
          if (i < g.I && (l & 15) < g.R) out[(int64_t)i * g.R + (l & 15)] = s;
        }
        __syncthreads();
      }
    }
  } else {
    // rows a, K-step of 4 rows
    // 64-wide i chunks per pass; NARROW launches (every I_n <= 64) need one
    constexpr int CHP = NARROW ? 1 : (sizeof(S) == 4 ? 4 : 2);
    const int64_t nsteps = (g.A + 3) / 4;
    const int64_t per_blk = (nsteps + mb.mblocks - 1) / mb.mblocks;
    const int64_t sbeg = (int64_t)blk * per_blk;
    const int64_t send = min(nsteps, sbeg + per_blk);
    const bool contig = (g.I % 4) == 0;
    const int nch = (g.I + 63) / 64;
    for (int c0 = 0; c0 < nch; c0 += CHP) {
      Acc acc[4][4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[c][t] = Acc{0, 0, 0, 0};
      if (contig) {
        // unconditional loads: row a clamped to A-1, chunk start clamped to
        // I-4, P_n row clamped to R-1, all masked
        for (int64_t st = sbeg + wave; st < send; st += kMWaves) {
          const int64_t a = st * 4 + q;
          const bool aok = a < g.A;
          const int64_t ac = aok ? a : g.A - 1;
          const S pv0 = gld<S>(mb.P + (int64_t)min(p, g.R - 1) * g.J + ac);
          V dv[CHP], yv[CHP];
#pragma unroll
          for (int c = 0; c < CHP; ++c) {
            const int i = min((c0 + c) * 64 + 4 * p, g.I - 4);
            dv[c] = gld<V>(pb.D + ac * g.I + i);
            yv[c] = gld<V>(mb.Y + ac * g.I + i);
          }
          // every load of the step is in flight before the first use
          __builtin_amdgcn_sched_barrier(0);
          const S pv = (aok && p < g.R) ? pv0 : S(0);
#pragma unroll
          for (int c = 0; c < CHP; ++c) {
            // chunks past I (the last pass) compute on zeros, no branch
            const bool ok = (c0 + c) * 64 + 4 * p < g.I;
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[c][t] = mma_op<BF, S>((ok ? dv[c][t] + yv[c][t] * inv_mu : S(0)), (pv), acc[c][t]);
          }
        }
      } else {
        for (int64_t st = sbeg + wave; st < send; st += kMWaves) {
          const int64_t a = st * 4 + q;
          const bool aok = a < g.A;
          const S pv = (aok && p < g.R) ? mb.P[(int64_t)p * g.J + a] : S(0);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (c >= CHP || c0 + c >= nch) break;
            const int i = (c0 + c) * 64 + 4 * p;
            const int nv = max(0, min(4, g.I - i));
            S gv[4] = {0, 0, 0, 0};
            if (aok && nv > 0) {
              int64_t o[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) o[t] = a * g.I + i + t;
              load_g4<S>(pb.D, mb.Y, o, contig, nv, inv_mu, gv);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[c][t] = mma_op<BF, S>((gv[t]), (pv), acc[c][t]);
          }
        }
      }
      for (int c = 0; c < 4; ++c) {
        if (c >= CHP || c0 + c >= nch) break;
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int v = 0; v < 4; ++v) red[wave][lane][v] = (double)acc[c][t][v];
          __syncthreads();
          if (threadIdx.x < 256) {
            const int l = threadIdx.x >> 2, v = threadIdx.x & 3;
            double s = 0;
#pragma unroll
            for (int w = 0; w < kMWaves; ++w) s += red[w][l][v];
            // D[m = row(l>>4, v)][n = l&15] -> i = 64(c0+c) + 4m + t
            const int m = MM<S>::row(l >> 4, v);
            const int i = (c0 + c) * 64 + 4 * m + t;
            if (i < g.I && (l & 15) < g.R) out[(int64_t)i * g.R + (l & 15)] = s;
          }
          __syncthreads();
        }
      }
    }
  }
}

// A mode whose GEMM-M the fused pass folds in (n < Problem::mmerge): M[i][r]
// is the sum over the fused blocks of every slab with index i, blocks
// (a I + i) K + k for term t = a K + k (a < A, k < K = mslab[n]); thread group
// grp sums the terms grp, grp + 4, ... of entry e = i R + r into
// acc[(t / 4) % 4], 16 loads in flight.
template <typename S>
__device__ __forceinline__ void merged_terms(const Problem<S>& pb, int n, int64_t e, int grp,
                                             double (&acc)[4]) {
  const ModeGeom g = pb.g[n];
  if (e >= (int64_t)g.I * g.R) return;
  const double* Mf = pb.m[n].Mf;
  const int64_t i = e / g.R, r = e - i * g.R;
  const int64_t K = pb.mslab[n], nt = g.A * K;
  constexpr int kRM = 16;
  for (int64_t t0 = grp; t0 < nt; t0 += 4 * kRM) {
    double v[kRM];
#pragma unroll
    for (int u = 0; u < kRM; ++u) {
      const int64_t t = t0 + 4 * u < nt ? t0 + 4 * u : nt - 1;
      const int64_t a = t / K, k = t - a * K;
      v[u] = Mf[((a * g.I + i) * K + k) * kRT + r];
    }
#pragma unroll
    for (int u = 0; u < kRM; ++u)
      if (t0 + 4 * u < nt) acc[u % 4] += v[u];
  }
}

// Fixed-order reduction of the GEMM-M partials: M[i][r] = sum_blk Mpart[blk][i][r]
// (partials I x R, the reduced M in rows of kRT whose columns >= R are unused).
// A block owns 64 consecutive entries; its 4 thread groups sum interleaved
// partials with independent loads in flight, then combine in a fixed order.
template <typename S>
__global__ void __launch_bounds__(256) k_reduce_m(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_REDUCE_M], pb.N, lb);
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int grp = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)(lb - pb.kb[KB_REDUCE_M][n]) * 64 + l;
  const int64_t ne = (int64_t)g.I * g.R;
  __shared__ double part[4][64];
  double acc[4] = {0, 0, 0, 0};
  if (n < pb.mmerge) {
    merged_terms<S>(pb, n, e, grp, acc);
  } else if (e < ne) {
    // group grp sums partials grp, grp + 4, ... into acc[(b / 4) % 4]; kRM
    // unconditional loads per pass (index clamped, value masked) are in
    // flight together
    constexpr int kRM = 24;
    const double* src = mb.Mpart + e;
    const int nb = mb.mblocks;
    for (int b0 = grp; b0 < nb; b0 += 4 * kRM) {
      double v[kRM];
#pragma unroll
      for (int u = 0; u < kRM; ++u) {
        const int b = b0 + 4 * u;
        v[u] = src[(int64_t)(b < nb ? b : nb - 1) * ne];
      }
#pragma unroll
      for (int u = 0; u < kRM; ++u)
        if (b0 + 4 * u < nb) acc[u % 4] += v[u];
    }
  }
  part[grp][l] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (grp == 0 && e < ne) {
    const int64_t i = e / g.R;
    mb.M[i * kRT + (e - i * g.R)] = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
  }
}

// The GEMM-M reduction of a problem whose fused pass accumulates every mode
// (Problem::mfull), in place of GEMM-M and k_reduce_m.  A merged mode's block
// adds its 64 entries' slab sums as k_reduce_m does.  For the fast modes the
// pass leaves one I_n x R partial per block in Mq; block (tile, q) of mode n
// takes the 64 entries e = 64 tile + lane, and its thread group grp the fused
// blocks of group g = 4 q + grp (the g-th of kMsumGroups runs of consecutive
// blocks), summed in block order with 16 loads in flight, into Mpart[g][e].
// The last of the tile's blocks to finish adds the kMsumGroups group sums in a
// fixed order into M (group grp the groups grp, grp + 4, ..., then the four in
// order).  The group sums, the count and the last block's reads are
// device-scope accesses, coherent across XCDs without a cache write-back, and
// a block's group sums are written (vmcnt(0)) before the barrier after which
// it counts itself.  (With a __threadfence() before each block counts itself
// this kernel took 37 us instead of 13 us.)
template <typename S>
__global__ void __launch_bounds__(256) k_msum(Batch<S> bt) {
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done || pb.sc->k == 0) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_MSUM], pb.N, lb);
  const int blk = lb - pb.kb[KB_MSUM][n];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int64_t ne = (int64_t)g.I * g.R;
  const int grp = threadIdx.x >> 6, l = threadIdx.x & 63;
  __shared__ double part[4][64];
  __shared__ int last;
  if (n < pb.mmerge) {
    const int64_t e = (int64_t)blk * 64 + l;
    double acc[4] = {0, 0, 0, 0};
    merged_terms<S>(pb, n, e, grp, acc);
    part[grp][l] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (grp == 0 && e < ne) {
      const int64_t i = e / g.R;
      mb.M[i * kRT + (e - i * g.R)] = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
    }
    return;
  }
  const int tiles = (int)((ne + 63) / 64);
  const int tile = blk % tiles, q = blk / tiles;
  const int gi = 4 * q + grp;
  const int64_t e = (int64_t)tile * 64 + l;
  const int nb = pb.fused_blocks;
  const int per = (nb + kMsumGroups - 1) / kMsumGroups;
  const int b0 = gi * per, b1 = min(nb, b0 + per);
  constexpr int kU = 16;
  if (e < ne) {
    double acc = 0.0;
    for (int bb = b0; bb < b1; bb += kU) {
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int b = bb + u < b1 ? bb + u : b1 - 1;
        v[u] = mb.Mq[(int64_t)b * ne + e];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (bb + u < b1) acc += v[u];
    }
    __hip_atomic_store(&mb.Mpart[(int64_t)gi * ne + e], acc, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this thread's group sum is written
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&mb.mcnt[tile], 1u, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) == (unsigned)(kMsumGroups / 4 - 1);
  __syncthreads();
  if (!last) return;
  if (threadIdx.x == 0)
    __hip_atomic_store(&mb.mcnt[tile], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double acc = 0.0;
  if (e < ne) {
    constexpr int kG = kMsumGroups / 4;
    double v[kG];
#pragma unroll
    for (int u = 0; u < kG; ++u)
      v[u] = __hip_atomic_load(&mb.Mpart[(int64_t)(grp + 4 * u) * ne + e], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int u = 0; u < kG; ++u) acc += v[u];
  }
  part[grp][l] = acc;
  __syncthreads();
  if (grp == 0 && e < ne) {
    const int64_t i = e / g.R;
    mb.M[i * kRT + (e - i * g.R)] = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
  }
}

// ---------------------------------------------------------------------------
// Gram S = P P^T in FP64 on the f64 MFMA: lane (p, q) holds P[p][c0+4q .. +3];
// A[m][k] = P[m][col], B[k][n] = P[n][col] are the same register.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_gram(Batch<S> bt) {
  typedef typename MM<S>::vec_t V;
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_GRAM], pb.N, lb);
  const int blk = lb - pb.kb[KB_GRAM][n];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  __shared__ double red[4][64][4];
  const int64_t nsteps = (g.J + 15) / 16;
  const int64_t per_blk = (nsteps + mb.sblocks - 1) / mb.sblocks;
  const int64_t sbeg = (int64_t)blk * per_blk;
  const int64_t send = min(nsteps, sbeg + per_blk);
  const bool pvec = (g.J % 4) == 0;
  d4v acc = d4v{0, 0, 0, 0};
  // full 16-column steps: unconditional vector loads of row p, kGramU steps of this wave per pass with all their loads
  // issued before the first MFMA
  constexpr int kGramU = 8;
  const int64_t full_end = pvec ? min(send, g.J / 16) : sbeg;
  // (lanes p >= R read row R-1, in cache anyway, and use zero)
  const bool pok = p < g.R;
  const S* prow = mb.P + (int64_t)min(p, g.R - 1) * g.J + 4 * q;
  // batches of 32 steps: the wave takes two runs of 4 consecutive steps, so
  // every row of P_n is read in 256-byte pieces
  int64_t bst = sbeg;
  for (; bst + 4 * kGramU <= full_end; bst += 4 * kGramU) {
    V v[kGramU];
#pragma unroll
    for (int u = 0; u < kGramU; ++u)
      v[u] = *reinterpret_cast<const V*>(prow + (bst + 16 * (u >> 2) + 4 * wave + (u & 3)) * 16);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kGramU; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double x = pok ? (double)v[u][t] : 0.0;
        acc = mma64(x, x, acc);
      }
  }
  int64_t st = bst + wave;
  for (; st < full_end; st += 4) {
    const V v = *reinterpret_cast<const V*>(prow + st * 16);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double x = pok ? (double)v[t] : 0.0;
      acc = mma64(x, x, acc);
    }
  }
  for (; st < send; st += 4) {
    const int64_t j4 = st * 16 + 4 * q;
    double pv[4] = {0, 0, 0, 0};
    if (p < g.R) {
      const S* prow = mb.P + (int64_t)p * g.J;
      if (pvec && j4 + 4 <= g.J) {
        V v = *reinterpret_cast<const V*>(prow + j4);
#pragma unroll
        for (int t = 0; t < 4; ++t) pv[t] = (double)v[t];
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) pv[t] = (j4 + t < g.J) ? (double)prow[j4 + t] : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = mma64(pv[t], pv[t], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][lane][v] = acc[v];
  __syncthreads();
  if (wave == 0) {
    double* out = mb.Spart + (int64_t)blk * kRT * kRT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double s = red[0][lane][v] + red[1][lane][v] + red[2][lane][v] + red[3][lane][v];
      out[MM<double>::row(q, v) * kRT + p] = s;  // S[row][p]
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// The Gram partials of a problem with some R_n > kRT: S_n = P_n P_n^T with P_n
// of T rank tiles, tile pair (a, b), a <= b, on FP64 MFMAs whose operands are
// the same lane fragments as in k_gram (lane (p, q) holds row kRT t + p at
// columns 4 q .. 4 q + 3 of the 16-column step), so tile a's fragment is A and
// tile b's is B.  Wave w takes steps w, w + 4, ...; the waves' sums are added
// in LDS in a fixed order, one tile pair at a time; the partial is RT x RT with
// both triangles written.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) k_gram_w(Batch<S> bt) {
  typedef typename MM<S>::vec_t V;
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_GRAM], pb.N, lb);
  const int blk = lb - pb.kb[KB_GRAM][n];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int T = g.T, RT = T * kRT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, q = lane >> 4;
  __shared__ double red[4][64][4];
  const int64_t nsteps = (g.J + 15) / 16;
  const int64_t per_blk = (nsteps + mb.sblocks - 1) / mb.sblocks;
  const int64_t sbeg = (int64_t)blk * per_blk;
  const int64_t send = min(nsteps, sbeg + per_blk);
  const bool pvec = (g.J % 4) == 0;
  constexpr int kPairs = kMaxTiles * (kMaxTiles + 1) / 2;
  d4v acc[kPairs];
#pragma unroll
  for (int e = 0; e < kPairs; ++e) acc[e] = d4v{0, 0, 0, 0};
  const S* prow[kMaxTiles];
  bool pok[kMaxTiles];
#pragma unroll
  for (int t = 0; t < kMaxTiles; ++t) {
    const int row = kRT * t + p;
    pok[t] = t < T && row < g.R;
    prow[t] = mb.P + (int64_t)min(row, g.R - 1) * g.J;
  }
  for (int64_t st = sbeg + wave; st < send; st += 4) {
    const int64_t j4 = st * 16 + 4 * q;
    const bool full = pvec && st * 16 + 16 <= g.J;
    double x[kMaxTiles][4];
#pragma unroll
    for (int t = 0; t < kMaxTiles; ++t) {
      if (full) {
        const V v = *reinterpret_cast<const V*>(prow[t] + j4);
#pragma unroll
        for (int u = 0; u < 4; ++u) x[t][u] = (double)v[u];
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) x[t][u] = j4 + u < g.J ? (double)prow[t][j4 + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) x[t][u] = pok[t] ? x[t][u] : 0.0;
    }
    int e = 0;
#pragma unroll
    for (int a = 0; a < kMaxTiles; ++a)
#pragma unroll
      for (int b = a; b < kMaxTiles; ++b, ++e)
        if (b < T) {
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[e] = mma64(x[a][u], x[b][u], acc[e]);
        }
  }
  double* out = mb.Spart + (int64_t)blk * RT * RT;
  int e = 0;
#pragma unroll
  for (int a = 0; a < kMaxTiles; ++a)
#pragma unroll
    for (int b = a; b < kMaxTiles; ++b, ++e) {
      if (b >= T) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wave][lane][v] = acc[e][v];
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double sm = red[0][lane][v] + red[1][lane][v] + red[2][lane][v] + red[3][lane][v];
          const int r = kRT * a + MM<double>::row(q, v), c = kRT * b + p;
          out[(int64_t)r * RT + c] = sm;  // S[r][c]
          if (a != b) out[(int64_t)c * RT + r] = sm;
        }
      }
      __syncthreads();
    }
}

int gemm_m_blocks(const ModeGeom& g, int N) {
  // one block of 8 waves per compute unit across the N modes of a solve (a
  // block holds its CU's register file), capped by the available K-steps
  const int64_t steps = g.B > 1 ? (g.J + 15) / 16 : (g.A + 3) / 4;
  // modes of at most 64 rows: four blocks per compute unit (one block's
  // waves hold too few loads in flight when each step covers only 4 row
  // blocks; measured at 64^4)
  const int64_t want = std::max(16, (g.I <= 64 ? 4 : 1) * kCUs / std::max(1, N));
  const int64_t maxb = (steps + kMWaves - 1) / kMWaves;
  return (int)std::max<int64_t>(1, std::min(want, maxb));
}

int gram_blocks(const ModeGeom& g) {
  // at most 64: the eigensolver loads every partial in one pass; 16 with more
  // than one rank tile (partials of RT x RT)
  const int64_t steps = (g.J + 15) / 16;
  int64_t want = g.T > 1 ? 16 : 64;
  int64_t maxb = (steps + 3) / 4;
  return (int)std::max<int64_t>(1, std::min(want, maxb));
}

int gemm_p_blocks(const ModeGeom& g) {
  if (g.B > 1 && g.B % 256 == 0) return (int)(g.J / 256);
  return (int)(g.B > 1 ? (g.J + 63) / 64 : (g.A + 63) / 64);
}

int reduce_m_blocks(const ModeGeom& g) { return (int)(((int64_t)g.I * g.R + 63) / 64); }

int msum_blocks(const ModeGeom& g) {
  return (int)(((int64_t)g.I * g.R + 63) / 64) * (kMsumGroups / 4);
}

template <typename S>
static int mode_grid(const Problem<S>& p, int kind) { return p.kb[kind][p.N]; }

// A set is homogeneous in precision (the batch driver groups by it); the
// BF16-input variant exists for the FP32 state only.
template <typename S>
static bool bf16_set(const LaunchSet<S>& ls) {
  return sizeof(S) == 4 && ls.host[0]->precision == PASD_BF16_GEMM;
}

// The unfolding GEMMs and the GEMM-M reduction work on one rank tile: a
// problem with some R_n > kRT enters as its tile views.  A set longer than
// kMaxBatch goes out in several launches.
template <typename S, typename F>
static void for_tile_sets(const LaunchSet<S>& ls, F launch) {
  LaunchSet<S> out;
  out.count = 0;
  for (int r = 0; r < ls.count; ++r) {
    const Problem<S>* h = ls.host[r];
    const int nv = h->wide ? h->ntiles : 1;
    for (int t = 0; t < nv; ++t) {
      if (out.count == kMaxBatch) {
        launch(out);
        out.count = 0;
      }
      out.host[out.count] = h->wide ? h->view_host[t] : h;
      out.dev[out.count] = h->wide ? h->view_dev[t] : ls.dev[r];
      ++out.count;
    }
  }
  if (out.count) launch(out);
}

template <typename S>
static void launch_gemm_p_set(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int tot = make_batch(ls, b, [](const Problem<S>& p) { return mode_grid(p, KB_GEMM_P); });
  LaunchSet<S> pair;
  pair.count = 0;
  for (int r = 0; r < ls.count; ++r)
    if (ls.host[r]->gp2) {
      pair.host[pair.count] = ls.host[r];
      pair.dev[pair.count] = ls.dev[r];
      ++pair.count;
    }
  Batch<S> b2;
  const int tot2 = pair.count ? make_batch(pair, b2, [](const Problem<S>& p) { return p.gp2; }) : 0;
  if constexpr (sizeof(S) == 4) {
    if (bf16_set(ls)) {
      if (tot) hipLaunchKernelGGL((k_gemm_p<S, true>), dim3(tot), dim3(256), 0, s, b);
      if (tot2) hipLaunchKernelGGL((k_gemm_p2<S, true>), dim3(tot2), dim3(256), 0, s, b2);
      return;
    }
  }
  // Order of the two launches, measured at 64^4: the pair first is faster with an
  // FP32 state (GEMM-P 81.7 -> 79.5 us) and slower in FP64 (195.5 -> 199.5 us).
  const bool pair_first = sizeof(S) == 4;
  if (pair_first && tot2) hipLaunchKernelGGL((k_gemm_p2<S, false>), dim3(tot2), dim3(256), 0, s, b2);
  if (tot) hipLaunchKernelGGL((k_gemm_p<S, false>), dim3(tot), dim3(256), 0, s, b);
  if (!pair_first && tot2) hipLaunchKernelGGL((k_gemm_p2<S, false>), dim3(tot2), dim3(256), 0, s, b2);
}

template <typename S>
void launch_gemm_p(const LaunchSet<S>& ls, hipStream_t s) {
  if (ls.count <= kMaxBatch && !any_wide(ls)) return launch_gemm_p_set(ls, s);
  for_tile_sets(ls, [s](const LaunchSet<S>& t) { launch_gemm_p_set(t, s); });
}

template <typename S>
static void launch_gemm_m_set(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int tot = make_batch(ls, b, [](const Problem<S>& p) { return mode_grid(p, KB_GEMM_M); });
  const bool one = ls.count == 1;
  // every mode of every problem at most 64 rows: the narrow instantiation
  bool narrow = true;
  for (int r = 0; r < ls.count; ++r)
    for (int n = 0; n < ls.host[r]->N; ++n) narrow = narrow && ls.host[r]->g[n].I <= 64;
  if constexpr (sizeof(S) == 4) {
    if (bf16_set(ls)) {
      if (narrow)
        hipLaunchKernelGGL((k_gemm_m<S, true, false, true>), dim3(tot), dim3(64 * kMWaves), 0, s, b);
      else if (one)
        hipLaunchKernelGGL((k_gemm_m<S, true, true, false>), dim3(tot), dim3(64 * kMWaves), 0, s, b);
      else
        hipLaunchKernelGGL((k_gemm_m<S, true, false, false>), dim3(tot), dim3(64 * kMWaves), 0, s, b);
      return;
    }
  }
  if (narrow)
    hipLaunchKernelGGL((k_gemm_m<S, false, false, true>), dim3(tot), dim3(64 * kMWaves), 0, s, b);
  else if (one)
    hipLaunchKernelGGL((k_gemm_m<S, false, true, false>), dim3(tot), dim3(64 * kMWaves), 0, s, b);
  else
    hipLaunchKernelGGL((k_gemm_m<S, false, false, false>), dim3(tot), dim3(64 * kMWaves), 0, s, b);
}

template <typename S>
void launch_gemm_m(const LaunchSet<S>& ls, hipStream_t s) {
  // problems whose fused pass accumulates every mode's M_n take the first
  // stage of its reduction instead (never wide: their ranks fit one tile)
  LaunchSet<S> full, rest;
  full.count = rest.count = 0;
  for (int r = 0; r < ls.count; ++r) {
    LaunchSet<S>& d = ls.host[r]->mfull ? full : rest;
    d.host[d.count] = ls.host[r];
    d.dev[d.count] = ls.dev[r];
    ++d.count;
  }
  if (full.count) {
    Batch<S> b;
    const int tot = make_batch(full, b, [](const Problem<S>& p) { return mode_grid(p, KB_MSUM); });
    hipLaunchKernelGGL(k_msum<S>, dim3(tot), dim3(256), 0, s, b);
  }
  if (!rest.count) return;
  if (rest.count <= kMaxBatch && !any_wide(rest)) return launch_gemm_m_set(rest, s);
  for_tile_sets(rest, [s](const LaunchSet<S>& t) { launch_gemm_m_set(t, s); });
}

template <typename S>
static void launch_reduce_m_set(const LaunchSet<S>& ls, hipStream_t s) {
  Batch<S> b;
  const int tot = make_batch(ls, b, [](const Problem<S>& p) { return mode_grid(p, KB_REDUCE_M); });
  hipLaunchKernelGGL(k_reduce_m<S>, dim3(tot), dim3(256), 0, s, b);
}

template <typename S>
void launch_reduce_m(const LaunchSet<S>& ls, hipStream_t s) {
  // k_msum has reduced every mode of the problems that fold them all
  LaunchSet<S> rest;
  rest.count = 0;
  for (int r = 0; r < ls.count; ++r) {
    if (ls.host[r]->mfull) continue;
    rest.host[rest.count] = ls.host[r];
    rest.dev[rest.count] = ls.dev[r];
    ++rest.count;
  }
  if (!rest.count) return;
  if (rest.count <= kMaxBatch && !any_wide(rest)) return launch_reduce_m_set(rest, s);
  for_tile_sets(rest, [s](const LaunchSet<S>& t) { launch_reduce_m_set(t, s); });
}

// ---------------------------------------------------------------------------
// Gram S = P P^T on the vector ALUs for ranks up to 8: each thread takes
// 16-byte chunks of columns of P_n (4 floats or 2 doubles), UR chunks per
// pass with every load in flight, and accumulates the upper triangle of the
// outer products in FP64 registers.  The block reduces them in a fixed order:
// within each 16-lane row by DPP exchanges (lanes i^1, i^2, then the mirror
// images within 8 and within 16 lanes; a + b and b + a round alike, so every
// lane of a row ends with the same row sum), then the 16 row sums of the
// block in LDS, in row order.  At these ranks the 16-wide FP64 MFMA tile of
// k_gram spends most of its work on padding and waits for its loads once per
// round of products (64^4, R_n = 6: FP64 24.6 -> 17.1 us, FP32 22.8 -> 13.3
// us); at R_n = 10 the MFMA kernel is the faster one (9.7 against 11.4 us at
// 200^3 FP32).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void row_sums(double (&acc)[NT]) {
  double t[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppXor1>(acc[e]);
#pragma unroll
  for (int e = 0; e < NT; ++e) acc[e] += t[e];
#pragma unroll
  for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppXor2>(acc[e]);
#pragma unroll
  for (int e = 0; e < NT; ++e) acc[e] += t[e];
#pragma unroll
  for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppHalfMirror>(acc[e]);
#pragma unroll
  for (int e = 0; e < NT; ++e) acc[e] += t[e];
#pragma unroll
  for (int e = 0; e < NT; ++e) t[e] = dpp_f64<kDppMirror>(acc[e]);
#pragma unroll
  for (int e = 0; e < NT; ++e) acc[e] += t[e];
}

template <typename S, int RP>
__global__ void __launch_bounds__(256) k_gram_v(Batch<S> bt) {
  typedef S v16 __attribute__((ext_vector_type(16 / sizeof(S))));
  constexpr int W = 16 / sizeof(S);
  constexpr int NT = RP * (RP + 1) / 2;
  constexpr int UR = (RP * W * sizeof(S) / 4 <= 24) ? 4 : 2;  // chunks per pass
  const int req = batch_find(bt.start, bt.nreq, blockIdx.x);
  const Problem<S>& pb = *bt.p[req];
  if (pb.sc->done) return;
  const int lb = blockIdx.x - bt.start[req];
  const int n = mode_of(pb.kb[KB_GRAM], pb.N, lb);
  const int blk = lb - pb.kb[KB_GRAM][n];
  const ModeGeom g = pb.g[n];
  const ModeBufs<S> mb = pb.m[n];
  const int R = g.R;
  const int64_t nch = (g.J + W - 1) / W;
  const int64_t per = (nch + mb.sblocks - 1) / mb.sblocks;
  const int64_t q0 = (int64_t)blk * per, q1 = min(nch, q0 + per);
  const bool vec = (g.J % W) == 0;
  double acc[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) acc[e] = 0.0;
  const PASD_GLOBAL S* rows[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r)
    rows[r] = (const PASD_GLOBAL S*)(mb.P + (int64_t)(r < R ? r : R - 1) * g.J);
  for (int64_t qb = q0 + threadIdx.x; qb < q1; qb += 256 * UR) {
    S x[UR][RP][W];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int64_t q = qb + 256 * u;
      const int64_t qc = q < q1 ? q : q0;  // clamped, masked below
      if (vec) {
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          const v16 v = *(const PASD_GLOBAL v16*)(rows[r] + qc * W);
#pragma unroll
          for (int t = 0; t < W; ++t) x[u][r][t] = v[t];
        }
      } else {
#pragma unroll
        for (int r = 0; r < RP; ++r)
#pragma unroll
          for (int t = 0; t < W; ++t) {
            const int64_t j = qc * W + t;
            x[u][r][t] = rows[r][j < g.J ? j : g.J - 1];
          }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int64_t q = qb + 256 * u;
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const bool ok = q < q1 && q * W + t < g.J;
        double xv[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) xv[r] = (ok && r < R) ? (double)x[u][r][t] : 0.0;
        int e = 0;
#pragma unroll
        for (int r = 0; r < RP; ++r)
#pragma unroll
          for (int c = r; c < RP; ++c, ++e) acc[e] = fma(xv[r], xv[c], acc[e]);
      }
    }
  }
  row_sums<NT>(acc);
  __shared__ double red[16][NT];
  if ((threadIdx.x & 15) == 0) {
#pragma unroll
    for (int e = 0; e < NT; ++e) red[threadIdx.x >> 4][e] = acc[e];
  }
  __syncthreads();
  {
    // entry (r, c) of the 16 x 16 partial, both triangles
    const int r = threadIdx.x / kRT, c = threadIdx.x % kRT;
    const int lo = r < c ? r : c, hi = r < c ? c : r;
    double v = 0.0;
    if (hi < RP) {
      const int e = lo * RP - lo * (lo - 1) / 2 + (hi - lo);
#pragma unroll
      for (int w = 0; w < 16; ++w) v += red[w][e];
    }
    mb.Spart[(int64_t)blk * kRT * kRT + threadIdx.x] = v;
  }
}

template <typename S>
void launch_gram(const LaunchSet<S>& ls, hipStream_t s) {
  LaunchSet<S> nar, wid;
  split_wide(ls, nar, wid);
  Batch<S> b;
  // problems whose ranks are all at most 8 take the vector-ALU Gram (the
  // choice is per problem, so a solve's partials are the same alone and in a
  // batch); the others the FP64 MFMA one
  LaunchSet<S> v, m;
  v.count = m.count = 0;
  int rv = 1;
  for (int r = 0; r < nar.count; ++r) {
    int rm = 1;
    for (int n = 0; n < nar.host[r]->N; ++n) rm = std::max(rm, nar.host[r]->g[n].R);
    LaunchSet<S>& d = rm <= 8 ? v : m;
    if (rm <= 8) rv = std::max(rv, rm);
    d.host[d.count] = nar.host[r];
    d.dev[d.count] = nar.dev[r];
    ++d.count;
  }
  if (v.count) {
    const int tot = make_batch(v, b, [](const Problem<S>& p) { return mode_grid(p, KB_GRAM); });
    switch ((rv + 1) / 2) {
      case 1: hipLaunchKernelGGL((k_gram_v<S, 2>), dim3(tot), dim3(256), 0, s, b); break;
      case 2: hipLaunchKernelGGL((k_gram_v<S, 4>), dim3(tot), dim3(256), 0, s, b); break;
      case 3: hipLaunchKernelGGL((k_gram_v<S, 6>), dim3(tot), dim3(256), 0, s, b); break;
      default: hipLaunchKernelGGL((k_gram_v<S, 8>), dim3(tot), dim3(256), 0, s, b); break;
    }
  }
  if (m.count) {
    const int tot = make_batch(m, b, [](const Problem<S>& p) { return mode_grid(p, KB_GRAM); });
    hipLaunchKernelGGL(k_gram<S>, dim3(tot), dim3(256), 0, s, b);
  }
  if (wid.count) {
    const int tot = make_batch(wid, b, [](const Problem<S>& p) { return mode_grid(p, KB_GRAM); });
    hipLaunchKernelGGL(k_gram_w<S>, dim3(tot), dim3(256), 0, s, b);
  }
}

#define INST(S)                                                         \
  template void launch_gemm_p<S>(const LaunchSet<S>&, hipStream_t);     \
  template void launch_gemm_m<S>(const LaunchSet<S>&, hipStream_t);     \
  template void launch_reduce_m<S>(const LaunchSet<S>&, hipStream_t);   \
  template void launch_gram<S>(const LaunchSet<S>&, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace pasd
