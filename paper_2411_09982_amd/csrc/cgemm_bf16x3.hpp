// Batched complex GEMM with FP32 operands on the BF16 matrix cores (gfx950).
//
// Every FP32 operand value x is split into three BF16 parts, each rounded to
// nearest from what the previous ones leave: x = h + m + l exactly for normal
// numbers, with |m| <= 2^-9 |x| and |l| <= 2^-18 |x|.  A real product keeps the
// six part products down to order 2^-18 (l*h, h*l, m*m, m*h, h*m, h*h, in rising
// size); the three it drops (m*l, l*m, l*l) are below 2^-26 of |x||y|.  The part
// products are exact in FP32; each K step's part products are summed apart from
// the running sum (cmac3), which is rounded once per step, and the products run
// on 16x16x32 BF16 MFMA (FP32 accumulation) at 2.5 PFLOP/s instead of 157 TFLOP/s.
//
// Same parameters, tile mapping and epilogues as cgemm_kernel<float>.  Tiles sit
// in LDS as FP32 (k-major, double-buffered: one barrier per K step); each wave
// splits the fragments it reads (v_cvt_pk_bf16_f32 rounds two values at once),
// so the splitting runs on the vector ALU beside the wave's MFMAs.
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

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to nearest-even BF16 and packed (a in the low half).
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

// Three-way split of two values into packed (hi, mid, lo) pairs.
__device__ __forceinline__ void split2(float a, float b, unsigned& h, unsigned& m, unsigned& l) {
  h = pk_bf16(a, b);
  const float ra = a - __uint_as_float(h << 16), rb = b - __uint_as_float(h & 0xffff0000u);
  m = pk_bf16(ra, rb);
  const float sa = ra - __uint_as_float(m << 16), sb = rb - __uint_as_float(m & 0xffff0000u);
  l = pk_bf16(sa, sb);
}

// The re and im parts of eight consecutive complex values as split fragments:
// re[0..2] = (h, m, l) of the real parts, im[0..2] of the imaginary parts.
__device__ __forceinline__ void split_frag(const float2 (&v)[8], u32x4 (&re)[3], u32x4 (&im)[3]) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    unsigned h, m, l;
    split2(v[2 * w].x, v[2 * w + 1].x, h, m, l);
    re[0][w] = h;
    re[1][w] = m;
    re[2][w] = l;
    split2(v[2 * w].y, v[2 * w + 1].y, h, m, l);
    im[0][w] = h;
    im[1][w] = m;
    im[2][w] = l;
  }
}

// One K step (32 k) of the complex block products of one A block with TN B
// blocks, Re += Ar Br - Ai Bi and Im += Ar Bi + Ai Br, for split operands
// (h, m, l) with -Ai given as nai: six part products per real product.  Each
// part sum of the step goes to a fresh accumulator (the five small part products
// first, then hi * hi), which is added to the running sum once: the running sum
// is rounded once per K step instead of once per MFMA, so the accumulation error
// stays at or below that of the FP32 MFMA kernel.  The 2 TN part sums advance
// round robin, so that no MFMA waits for the one before it.
template <int TN>
__device__ __forceinline__ void cmac3(const u32x4 (&ar)[3], const u32x4 (&ai)[3], const u32x4 (&nai)[3],
                                      const u32x4 (&br)[TN][3], const u32x4 (&bi)[TN][3], f32x4 (&accr)[TN],
                                      f32x4 (&acci)[TN]) {
  f32x4 tr[TN], ti[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) tr[j] = ti[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int PX[6] = {2, 0, 1, 1, 0, 0}, PY[6] = {0, 2, 1, 0, 1, 0};   // lo*hi, hi*lo, mid*mid, mid*hi, hi*mid, hi*hi
#pragma unroll
  for (int t = 0; t < 6; ++t) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      tr[j] = mfma16_bf16(ar[PX[t]], br[j][PY[t]], tr[j]);
      ti[j] = mfma16_bf16(ar[PX[t]], bi[j][PY[t]], ti[j]);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      tr[j] = mfma16_bf16(nai[PX[t]], bi[j][PY[t]], tr[j]);
      ti[j] = mfma16_bf16(ai[PX[t]], br[j][PY[t]], ti[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      accr[j][e] += tr[j][e];
      acci[j][e] += ti[j][e];
    }
}

template <int BM, int BN, int WM, int WN, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void cgemm_bf16x3_kernel(
    GemmParams<float> p) {
  using C2 = float2;
  constexpr int BK = 32;        // one 16x16x32 instruction per K step
  constexpr int WAVES_N = BN / WN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert((BM / WM) * (BN / WN) * 64 == NT, "one wave per WM x WN sub-tile");
  static_assert(BM * (BK / 8) == NT && BN * (BK / 8) == NT, "each thread moves eight k values of A and of B");

  // k-major tiles, as in cgemm_kernel: a lane's eight k values of one row of A
  // (column of B) sit one LDS row apart, and the 16 lanes that read one k hit
  // consecutive addresses
  __shared__ __attribute__((aligned(16))) C2 As[2][BK][BM + 1];
  __shared__ __attribute__((aligned(16))) C2 Bs[2][BK][BN];

  TileJob<float> jb;
  if (!tile_job<float, BM, BN>(p, xcd_remap(blockIdx.x, gridDim.x), jb)) return;

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
  // The zero-select of out-of-range values waits for the store, so that no
  // instruction before the MFMAs depends on the loads in flight.
  C2 ra[8], rb[8];
  auto load = [&](int k0) {
    const int arow = min(jb.row0 + ar, p.M - 1) * lda;
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = jb.A[arow + max(0, min(k0 + ak + q, p.K - 1))];
    const int bcol = min(jb.col0 + bc, p.N - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      rb[q] = jb.B[max(0, min(k0 + bk + q, p.K - 1)) * ldb + bcol];
    }
  };
  auto store = [&](int buf, int k0) {
    const bool arow_in = jb.row0 + ar < p.M, bcol_in = jb.col0 + bc < p.N;
#pragma unroll
    for (int q = 0; q < 8; ++q) As[buf][ak + q][ar] = (arow_in && k0 + ak + q < p.K) ? ra[q] : czero<C2>();
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[buf][bk + q][bc] = (bcol_in && k0 + bk + q < p.K) ? rb[q] : czero<C2>();
  };

  const int nk = (p.K + BK - 1) / BK;
  if (nk > 0) {   // K = 0 (C = beta C + terms) reads no operand
    load(0);
    store(0, 0);
  }
  __syncthreads();
  const int fr = lane & 15, fk = 8 * (lane >> 4);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
    if (!idle) {
      u32x4 bre[TN][3], bim[TN][3];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        C2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = Bs[cur][fk + q][wn + j * 16 + fr];
        split_frag(v, bre[j], bim[j]);
      }
      // A fragments in a software pipeline: while the MFMAs of block i run, the
      // fragment of block i + 1 is read and split on the vector ALU, the two
      // streams interleaved instruction by instruction
      u32x4 are[3], aim[3];
      {
        C2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = As[cur][fk + q][wm + fr];
        split_frag(v, are, aim);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        C2 vn[8];
        if (i + 1 < TM) {
#pragma unroll
          for (int q = 0; q < 8; ++q) vn[q] = As[cur][fk + q][wm + (i + 1) * 16 + fr];
        }
        u32x4 naim[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) naim[pl] = aim[pl] ^ 0x80008000u;   // -Ai: flip the BF16 sign bits
        cmac3<TN>(are, aim, naim, bre, bim, accr[i], acci[i]);
        if (i + 1 < TM) {
          split_frag(vn, are, aim);
          // 24 TN MFMAs against about 90 VALU of the split: one MFMA, then two VALU
#pragma unroll
          for (int g = 0; g < 24 * TN; ++g) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
          }
        }
      }
    }
    if (kt + 1 < nk) store(cur ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

  tile_epilogue<float, TM, TN>(p, jb, accr, acci, wm, wn, lane);
}

// Variant that splits each value once per workgroup, as it is stored to LDS: the
// tile sits in LDS as six BF16 planes (re and im times hi, mid, lo) with k
// contiguous, each 16-byte chunk of a row at chunk index c ^ ((row >> 2) & 3) so
// that the 16 lanes reading one fragment hit 16 different bank groups.  One K
// step of planes takes 96 KB, so LDS holds one step; the next step's values wait
// in registers and are split and stored between two barriers after the MFMAs.
// The MFMA loop itself has no vector-ALU work but the sign flips of -Ai.
template <int BM, int BN, int WM, int WN, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void cgemm_bf16x3_planes_kernel(
    GemmParams<float> p) {
  using C2 = float2;
  constexpr int BK = 32;
  constexpr int WAVES_N = BN / WN;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert((BM / WM) * (BN / WN) * 64 == NT, "one wave per WM x WN sub-tile");
  static_assert(BM * (BK / 8) == NT && BN * (BK / 8) == NT, "each thread moves eight k values of A and of B");

  // [plane][row][k] as 16-byte chunks of eight BF16: row r, chunk c at index
  // r * 4 + (c ^ ((r >> 2) & 3))
  __shared__ u32x4 As[6][BM * (BK / 8)];
  __shared__ u32x4 Bs[6][BN * (BK / 8)];

  TileJob<float> jb;
  if (!tile_job<float, BM, BN>(p, xcd_remap(blockIdx.x, gridDim.x), jb)) return;

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

  const int ar = tid / (BK / 8), ak = (tid % (BK / 8)) * 8;
  const int bc = tid % BN, bk = (tid / BN) * 8;
  const int lda = int(p.lda), ldb = int(p.ldb);
  C2 ra[8], rb[8];
  auto load = [&](int k0) {
    const int arow = min(jb.row0 + ar, p.M - 1) * lda;
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = jb.A[arow + max(0, min(k0 + ak + q, p.K - 1))];
    const int bcol = min(jb.col0 + bc, p.N - 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      rb[q] = jb.B[max(0, min(k0 + bk + q, p.K - 1)) * ldb + bcol];
    }
  };
  auto chunk = [](int row, int c) { return row * (BK / 8) + (c ^ ((row >> 2) & 3)); };
  auto store = [&](int k0) {
    const bool arow_in = jb.row0 + ar < p.M, bcol_in = jb.col0 + bc < p.N;
    C2 va[8], vb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      va[q] = (arow_in && k0 + ak + q < p.K) ? ra[q] : czero<C2>();
      vb[q] = (bcol_in && k0 + bk + q < p.K) ? rb[q] : czero<C2>();
    }
    u32x4 re[3], im[3];
    split_frag(va, re, im);
    const int ca = chunk(ar, ak / 8);
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
      As[pl][ca] = re[pl];
      As[3 + pl][ca] = im[pl];
    }
    split_frag(vb, re, im);
    const int cb = chunk(bc, bk / 8);
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
      Bs[pl][cb] = re[pl];
      Bs[3 + pl][cb] = im[pl];
    }
  };

  const int nk = (p.K + BK - 1) / BK;
  if (nk > 0) {   // K = 0 (C = beta C + terms) reads no operand
    load(0);
    store(0);
  }
  __syncthreads();
  const int fr = lane & 15, fc = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * BK);
    if (!idle) {
      u32x4 bre[TN][3], bim[TN][3];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int cb = chunk(wn + j * 16 + fr, fc);
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
          bre[j][pl] = Bs[pl][cb];
          bim[j][pl] = Bs[3 + pl][cb];
        }
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int ca = chunk(wm + i * 16 + fr, fc);
        u32x4 are[3], aim[3], naim[3];
#pragma unroll
        for (int pl = 0; pl < 3; ++pl) {
          are[pl] = As[pl][ca];
          aim[pl] = As[3 + pl][ca];
          naim[pl] = aim[pl] ^ 0x80008000u;   // -Ai: flip the BF16 sign bits
        }
        cmac3<TN>(are, aim, naim, bre, bim, accr[i], acci[i]);
      }
    }
    if (kt + 1 < nk) {
      __syncthreads();   // every wave is done with this K step's planes
      store((kt + 1) * BK);
    }
    __syncthreads();
  }

  tile_epilogue<float, TM, TN>(p, jb, accr, acci, wm, wn, lane);
}

}  // namespace qcheff
