// Batched complex GEMM with FP32 operands on the BF16 matrix cores (gfx950).
//
// Every FP32 operand value x is split into three BF16 parts, each rounded to
// nearest from what the previous ones leave: x = h + m + l + r with |m| <= 2^-8 |x|,
// |l| <= 2^-16 |x| and |r| <= 2^-24 |x|.  A real product keeps the six part
// products down to order 2^-16 (l*h, h*l, m*m, m*h, h*m, h*h, in rising size);
// the three it drops (m*l, l*m, l*l) are below 2^-23 of |x||y|, so a sum of
// products is as accurate as FP32 arithmetic while it runs on 16x16x32 BF16
// MFMA (FP32 accumulation) at 2.5 PFLOP/s instead of FP32 MFMA at 157 TFLOP/s.
//
// Same parameters, tile mapping and epilogues as cgemm_kernel<float>.  The loader
// splits each value once as it moves a tile into LDS, where every operand is
// stored as six BF16 planes (re h, m, l; im h, m, l) with k contiguous, so that a
// lane reads the eight consecutive k values of one 16x16x32 fragment at once.
// LDS holds one K step (122 KB); the next is fetched into registers meanwhile.
#pragma once

#include "cgemm.hpp"

namespace qcheff {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// D = A(16x32) B(32x16) + C.  Lane l supplies A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i = 0..7; D is laid out as the FP32 16x16x4 result.
__device__ __forceinline__ f32x4 mfma16_bf16(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                  0, 0, 0);
}

// BF16 bits of x rounded to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ unsigned bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (x != x) ? 0x7fc0u : (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void split3(float x, unsigned& h, unsigned& m, unsigned& l) {
  h = bf16_rne(x);
  const float r1 = x - __uint_as_float(h << 16);
  m = bf16_rne(r1);
  const float r2 = r1 - __uint_as_float(m << 16);
  l = bf16_rne(r2);
}

// c += x y for split operands x = (h, m, l), y = (h, m, l): six part products,
// the smallest first.
__device__ __forceinline__ f32x4 prod3(const u32x4 (&x)[3], const u32x4 (&y)[3], f32x4 c) {
  c = mfma16_bf16(x[2], y[0], c);
  c = mfma16_bf16(x[0], y[2], c);
  c = mfma16_bf16(x[1], y[1], c);
  c = mfma16_bf16(x[1], y[0], c);
  c = mfma16_bf16(x[0], y[1], c);
  c = mfma16_bf16(x[0], y[0], c);
  return c;
}

template <int BM, int BN, int WM, int WN, int NT, bool BCOMB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void cgemm_bf16x3_kernel(
    GemmParams<float> p) {
  using C2 = float2;
  constexpr int BK = 32;        // one 16x16x32 instruction per K step
  constexpr int KP = BK + 8;    // LDS row: 32 BF16 padded to 80 bytes
  constexpr int WAVES_N = BN / WN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert((BM / WM) * (BN / WN) * 64 == NT, "one wave per WM x WN sub-tile");
  static_assert(BM * (BK / 8) == NT && BN * (BK / 8) == NT, "each thread moves eight k values of A and of B");

  __shared__ __attribute__((aligned(16))) unsigned short As[6][BM][KP];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[6][BN][KP];

  TileJob<float> jb;
  if (!tile_job<float, BM, BN>(p, jb)) return;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave / WAVES_N) * WM, wn = (wave % WAVES_N) * WN;
  const bool idle = p.herm && jb.tm == jb.tn && wm >= wn + WN;

  f32x4 accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) { accr[i][j][e] = 0.f; acci[i][j][e] = 0.f; }

  // Thread roles: row ar of A and column bc of B, eight consecutive k each.
  // Loads are unconditional (clamped addresses, zero-select), as in cgemm_kernel.
  const int ar = tid / (BK / 8), ak = (tid % (BK / 8)) * 8;
  const int bc = tid % BN, bk = (tid / BN) * 8;
  const int lda = int(p.lda), ldb = int(p.ldb);
  C2 ra[8], rb[8];
  auto load = [&](int k0) {
    const int gr = jb.row0 + ar;
    const int arow = min(gr, p.M - 1) * lda;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int gk = k0 + ak + q;
      const C2 v = jb.A[arow + max(0, min(gk, p.K - 1))];
      ra[q] = (gr < p.M && gk < p.K) ? v : czero<C2>();
    }
    const int gc = jb.col0 + bc;
    const int bcol = min(gc, p.N - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int gk = k0 + bk + q;
      const int off = max(0, min(gk, p.K - 1)) * ldb + bcol;
      C2 v = jb.B[off];
      if constexpr (BCOMB) {
        const C2 x0 = jb.BX0[off], x1 = jb.BX1[off];
        v.x = p.bxc[0] * v.x + p.bxc[1] * x0.x + p.bxc[2] * x1.x;
        v.y = p.bxc[0] * v.y + p.bxc[1] * x0.y + p.bxc[2] * x1.y;
      }
      rb[q] = (gk < p.K && gc < p.N) ? v : czero<C2>();
    }
  };
  // Split eight values into the six planes of one 16-byte LDS row segment.
  static_assert(BM == BN, "square tiles (the LDS planes of A and B share one shape)");
  auto split_store = [&](unsigned short (&S)[6][BM][KP], const C2 (&v)[8], int row, int k) {
    u32x4 pk[6];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      unsigned h0, m0, l0, h1, m1, l1;
      split3(v[2 * w].x, h0, m0, l0);
      split3(v[2 * w + 1].x, h1, m1, l1);
      pk[0][w] = h0 | (h1 << 16);
      pk[1][w] = m0 | (m1 << 16);
      pk[2][w] = l0 | (l1 << 16);
      split3(v[2 * w].y, h0, m0, l0);
      split3(v[2 * w + 1].y, h1, m1, l1);
      pk[3][w] = h0 | (h1 << 16);
      pk[4][w] = m0 | (m1 << 16);
      pk[5][w] = l0 | (l1 << 16);
    }
#pragma unroll
    for (int pl = 0; pl < 6; ++pl) *reinterpret_cast<u32x4*>(&S[pl][row][k]) = pk[pl];
  };
  auto store = [&]() {
    split_store(As, ra, ar, ak);
    split_store(Bs, rb, bc, bk);
  };

  const int nk = (p.K + BK - 1) / BK;
  if (nk > 0) {   // K = 0 (C = beta C + terms) reads no operand
    load(0);
    store();
  }
  __syncthreads();
  const int fr = lane & 15, fk = 8 * (lane >> 4);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * BK);
    if (!idle) {
      u32x4 bre[TN][3], bim[TN][3];
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
          bre[j][pl] = *reinterpret_cast<const u32x4*>(&Bs[pl][wn + j * 16 + fr][fk]);
          bim[j][pl] = *reinterpret_cast<const u32x4*>(&Bs[3 + pl][wn + j * 16 + fr][fk]);
        }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        u32x4 are[3], aim[3], naim[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
          are[pl] = *reinterpret_cast<const u32x4*>(&As[pl][wm + i * 16 + fr][fk]);
          aim[pl] = *reinterpret_cast<const u32x4*>(&As[3 + pl][wm + i * 16 + fr][fk]);
          naim[pl] = aim[pl] ^ 0x80008000u;   // -Ai: flip the BF16 sign bits
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          // Re += Ar Br - Ai Bi,  Im += Ar Bi + Ai Br
          accr[i][j] = prod3(are, bre[j], accr[i][j]);
          accr[i][j] = prod3(naim, bim[j], accr[i][j]);
          acci[i][j] = prod3(are, bim[j], acci[i][j]);
          acci[i][j] = prod3(aim, bre[j], acci[i][j]);
        }
      }
    }
    __syncthreads();   // every wave is done with this K step's planes
    if (kt + 1 < nk) {
      store();
      __syncthreads();
    }
  }

  tile_epilogue<float, TM, TN>(p, jb, accr, acci, wm, wn, lane);
}

}  // namespace qcheff
