// Batched complex GEMM on MFMA (gfx950), FP32 or FP64, interleaved complex storage.
//
//   C_b = alpha * A_b B_b + beta * C_b + sum_i xc[i] X_{i,b} + gamma * I      (EPI_STD)
//   aug_b[:, :N] = V_b - A_b B_b,  aug_b[:, off:off+N] = V_b + A_b B_b (FP64)  (EPI_AUG)
//   aug_b = X_{0,b} + alpha * A_b B_b, formed and written in FP64            (EPI_OUT64)
//   c32_b = EPI_STD's value, written in complex64                            (EPI_C32)
//
// The FP64 kernels with MODE 1 take complex64 operands A_b = R_b, B_b = R_b^dag
// (R = a32) and widen them to FP64 as they load: the products of FP32 values are
// exact in FP64, so R R^dag is formed to FP64 accuracy without an FP64 copy of R.
//
// A complex product is four real MFMA products on planar operands:
//   Re += Ar Br - Ai Bi,  Im += Ar Bi + Ai Br.
// A workgroup of NT / 64 waves owns a BM x BN tile of C; each wave a WM x WN
// sub-tile built from 16x16x4 MFMA instructions.  K advances BK at a time
// through double-buffered LDS; the next tile is fetched into registers while
// the current one is consumed.  Any M, N, K, leading dimension and offset is
// accepted: k past K reads as zero, rows of A past M and columns of B past N
// read a clamped valid element (they only feed outputs that are not stored),
// and out-of-range stores are skipped.
#pragma once

#include "common.hpp"

namespace qcheff {

enum { EPI_STD = 0, EPI_AUG = 1, EPI_OUT64 = 2, EPI_C32 = 3 };

// Kernel ids of the timing instrumentation (match QCHEFF_KERNEL_* in qcheff.h).
enum { KERNEL_GEMM_F32 = 1, KERNEL_GEMM_F64 = 2, KERNEL_GEMM_BF16X3 = 3, KERNEL_ACTION = 4 };

// Records a HIP event pair around a launch while timing is enabled.
struct LaunchTimer {
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  void begin(hipStream_t st);
  void end(hipStream_t st, int kernel, double flops, double bytes);
};

template <typename T> struct GemmParams {
  using C2 = typename Cx<T>::t;
  int M, N, K, batch;
  int tiles_m, tiles_n;
  const C2* A; int64_t lda, sA;
  const C2* B; int64_t ldb, sB;
  C2* C; int64_t ldc, sC;
  T alpha, beta, gamma;
  int cfg;                      // tile configuration (GemmTile<T, cfg>)
  int herm;                     // 0: general; +1 / -1: the result is Hermitian / skew-Hermitian
                                // (M == N, BM == BN): only the upper triangle of tiles runs
  int epi;                      // EPI_STD, EPI_AUG or EPI_OUT64
  int sq;                       // 1: squaring mode (sq_* fields)
  int nx;                       // number of X terms (0..3); X share C's ld and stride
  const C2* X[3]; T xc[3];
  // EPI_AUG / EPI_OUT64 target (FP64 always)
  double2* aug; int64_t ld_aug, s_aug, aug_off;
  // squaring mode: A = B = in, C = out, chosen per item from the remaining count
  const int* sq_s; int sq_step; C2* sq_p0; C2* sq_p1;
  // EPI_C32 target (ldc, sC)
  float2* c32;
  // mode 1 (FP64 kernels only): A = R, B = R^dag for the complex64 matrices R
  int mode;
  const float2* a32; int64_t ld32, s32;
};

// The item and tile a workgroup computes, and its operand pointers.
template <typename T> struct TileJob {
  using C2 = typename Cx<T>::t;
  int b, tm, tn, row0, col0;
  const C2* A;
  const C2* B;
  C2* C;
  const float2* R;   // mode 1: the item's complex64 operand
};

// Fills `j` for logical tile `bid` (item-major, then tile); false when it has
// nothing to do (past the last item, or an item whose squarings are done).
// With a (skew-)Hermitian result only the tiles on and above the diagonal run;
// each element above the diagonal is also written, conjugated, below it.
template <typename T, int BM, int BN>
__device__ __forceinline__ bool tile_job(const GemmParams<T>& p, int bid, TileJob<T>& j) {
  using C2 = typename Cx<T>::t;
  const int tiles = p.herm ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  const int b = bid / tiles;
  if (b >= p.batch) return false;
  const int t = bid - b * tiles;
  int tm, tn;
  if (p.herm) {
    tm = 0;
    int rem = t;
    while (rem >= p.tiles_m - tm) {
      rem -= p.tiles_m - tm;
      ++tm;
    }
    tn = tm + rem;
  } else {
    tm = t / p.tiles_n;
    tn = t % p.tiles_n;
  }
  j.b = b;
  j.tm = tm;
  j.tn = tn;
  j.row0 = tm * BM;
  j.col0 = tn * BN;
  if (p.sq) {
    const int s = p.sq_s[b];
    if (s <= p.sq_step) return false;        // this item needs no more squarings
    const int rem = s - p.sq_step;           // squarings left, this one included
    C2* in = (rem % 2 == 0) ? p.sq_p0 : p.sq_p1;
    C2* out = (rem % 2 == 0) ? p.sq_p1 : p.sq_p0;
    j.A = in + b * p.sA;
    j.B = in + b * p.sB;
    j.C = out + b * p.sC;
  } else {
    j.A = p.A + b * p.sA;
    j.B = p.B + b * p.sB;
    j.C = p.C + b * p.sC;
  }
  j.R = p.mode == 1 ? p.a32 + b * p.s32 : nullptr;
  return true;
}

// Writes a wave's TM x TN blocks of 16 x 16 accumulators (rows as acc_row<T>,
// column lane % 16) through the epilogue the parameters select.  The mirror
// half of a (skew-)Hermitian EPI_STD / EPI_C32 result goes through `scr`, the
// wave's 16 x 16 LDS block: written transposed, it is read back so that 16
// lanes store 16 consecutive elements of one row (written straight from the
// accumulators, each lane's four values would land in four rows).
template <typename T, int TM, int TN>
__device__ __forceinline__ void tile_epilogue(const GemmParams<T>& p, const TileJob<T>& jb,
                                              const typename Cx<T>::acc (&accr)[TM][TN],
                                              const typename Cx<T>::acc (&acci)[TM][TN], int wm, int wn,
                                              int lane, typename Cx<T>::t* scr = nullptr) {
  using C2 = typename Cx<T>::t;
  const int b = jb.b;
  C2* C = jb.C;
  const bool lds_mirror = scr && p.herm && (p.epi == EPI_STD || p.epi == EPI_C32);
  // (the LDS path for the augmented system's two FP64 mirrors fits the
  // registers of 32 x 32 wave tiles; larger ones store them directly)
  const bool aug_mirror = TM * TN <= 4 && scr && p.herm && p.epi == EPI_AUG;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = jb.col0 + wn + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = jb.row0 + wm + i * 16 + acc_row<T>(lane, e);
        if (r >= p.M || c >= p.N) continue;
        if (p.herm && r > c) continue;   // written as the mirror of (c, r)
        const int64_t off = int64_t(r) * p.ldc + c;
        if (p.epi == EPI_OUT64) {
          // a small correction added to X_0 in FP64: X_0's value is exact there
          const C2 xv = p.X[0][b * p.sC + off];
          p.aug[b * p.s_aug + int64_t(r) * p.ld_aug + c] =
              make_double2(double(xv.x) + double(p.alpha * accr[i][j][e]),
                           double(xv.y) + double(p.alpha * acci[i][j][e]));
        } else if (p.epi == EPI_AUG) {
          // U = A W is skew-Hermitian here and V Hermitian: q = V - U, p = V + U,
          // and below the diagonal q(c, r) = conj(p(r, c)), p(c, r) = conj(q(r, c))
          C2 v = p.X[0][b * p.sC + off];
          double pr = double(accr[i][j][e]), pi = double(acci[i][j][e]);
          if (p.herm && r == c) {
            v.y = T(0);
            pr = 0.0;
          }
          double2* base = p.aug + b * p.s_aug;
          const double2 q = make_double2(double(v.x) - pr, double(v.y) - pi);
          const double2 pp = make_double2(double(v.x) + pr, double(v.y) + pi);
          base[int64_t(r) * p.ld_aug + c] = q;
          base[int64_t(r) * p.ld_aug + p.aug_off + c] = pp;
          if (p.herm && r != c && !aug_mirror) {
            base[int64_t(c) * p.ld_aug + r] = make_double2(pp.x, -pp.y);
            base[int64_t(c) * p.ld_aug + p.aug_off + r] = make_double2(q.x, -q.y);
          }
        } else {
          T vr = p.alpha * accr[i][j][e], vi = p.alpha * acci[i][j][e];
          if (p.beta != T(0)) {
            const C2 old = C[off];
            vr += p.beta * old.x;
            vi += p.beta * old.y;
          }
          for (int x = 0; x < p.nx; ++x) {
            const C2 xv = p.X[x][b * p.sC + off];
            vr += p.xc[x] * xv.x;
            vi += p.xc[x] * xv.y;
          }
          if (r == c) vr += p.gamma;
          if (p.herm && r == c) {   // a Hermitian diagonal is real, a skew-Hermitian one imaginary
            if (p.herm > 0) vi = T(0); else vr = T(0);
          }
          if (p.epi == EPI_C32) {
            p.c32[b * p.sC + off] = make_float2(float(vr), float(vi));
          } else {
            C2 o;
            o.x = vr;
            o.y = vi;
            C[off] = o;
          }
          if (p.herm && r != c) {   // the value of (c, r)
            C2 m;
            m.x = p.herm > 0 ? vr : -vr;
            m.y = p.herm > 0 ? -vi : vi;
            const int64_t moff = int64_t(c) * p.ldc + r;
            if (lds_mirror)   // at the block's transposed place, stored below
              scr[(lane & 15) * 16 + (acc_row<T>(lane, e) ^ (lane & 15))] = m;
            else if (p.epi == EPI_C32)
              p.c32[b * p.sC + moff] = make_float2(float(m.x), float(m.y));
            else
              C[moff] = m;
          }
        }
      }
      if (lds_mirror) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int R0 = jb.row0 + wm + i * 16, C0 = jb.col0 + wn + j * 16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int tr = acc_row<T>(lane, e), tc = lane & 15;
          const int r = R0 + tc, c = C0 + tr;   // the element whose mirror lands at (c, r)
          const C2 m = scr[tr * 16 + (tc ^ tr)];
          if (r < c && r < p.M && c < p.N) {
            const int64_t moff = int64_t(c) * p.ldc + r;
            if (p.epi == EPI_C32)
              p.c32[b * p.sC + moff] = make_float2(float(m.x), float(m.y));
            else
              C[moff] = m;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      if constexpr (TM * TN <= 4) if (aug_mirror) {
        // the two FP64 mirrors, q(c, r) = conj(p(r, c)) and p(c, r) = conj(q(r, c)),
        // through 2 KB of the wave's LDS block (8 x 16 complex128) at a time: for
        // each value and each half of the block's columns, the lanes holding those
        // columns recompute it (V read again) and write it transposed, then all
        // lanes read back rows and store 16 consecutive elements of each
        double2* s2 = reinterpret_cast<double2*>(scr);
        const int R0 = jb.row0 + wm + i * 16, C0 = jb.col0 + wn + j * 16;
        double2* base = p.aug + b * p.s_aug;
        const int cl = lane & 15;
#pragma unroll
        for (int which = 0; which < 2; ++which) {   // 0: conj(p) into q's half, 1: conj(q) into p's
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if ((cl >> 3) == h) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int rl = acc_row<T>(lane, e);
                const int r = R0 + rl, c = C0 + cl;
                if (r >= p.M || c >= p.N || r >= c) continue;   // no mirror to write
                const C2 v = p.X[0][b * p.sC + int64_t(r) * p.ldc + c];
                const double pr = double(accr[i][j][e]), pi = double(acci[i][j][e]);
                const double2 m = which == 0 ? make_double2(double(v.x) + pr, -(double(v.y) + pi))
                                             : make_double2(double(v.x) - pr, -(double(v.y) - pi));
                s2[(cl - 8 * h) * 16 + (rl ^ (cl - 8 * h))] = m;
              }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const int tr = (lane >> 4) + 4 * k, tc = lane & 15;   // block column 8 h + tr, row tc
              const int r = R0 + tc, c = C0 + 8 * h + tr;           // the element whose mirror this is
              const double2 m = s2[tr * 16 + (tc ^ tr)];
              if (r < c && r < p.M && c < p.N)
                base[int64_t(c) * p.ld_aug + (which == 0 ? 0 : p.aug_off) + r] = m;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          }
        }
      }
    }
  }
}

// Sub-tile positions (row * 4 + column in a 4 x 4 grid) of the sixteen waves of
// a 16-wave tile, four bits per wave.  A workgroup's waves are dealt to the four
// SIMDs round-robin (waves w, w + 4, w + 8 and w + 12 share one; measured with
// the hardware id register), and in a diagonal tile of a (skew-)Hermitian result
// only the 10 positions on or above the diagonal do MFMA work.  In row-major
// order one SIMD would carry four busy waves and another one; in this order
// every SIMD carries two or three (so does every set {w : w / 4 = k}): +3-4 %
// on Hermitian-half products at d = 512-1024, general ones unchanged.  Which
// wave computes an element does not change how: results are the same bits.
constexpr uint64_t kWavePos16 = 0xEFADB3C5'78916420ull;

// One tile of C through the K loop and the epilogue (the LDS buffers belong to
// the calling kernel).
template <typename T, int BM, int BN, int BK, int WM, int WN, int NT, int MODE>
__device__ __forceinline__ void cgemm_tile(const GemmParams<T>& p, const TileJob<T>& jb,
                                           typename Cx<T>::t (&As)[2][BK][BM + 1],
                                           typename Cx<T>::t (&Bs)[2][BK][BN + (MODE == 1)]) {
  using C2 = typename Cx<T>::t;
  using Acc = typename Cx<T>::acc;
  constexpr int WAVES_N = BN / WN;
  static_assert((BM / WM) * (BN / WN) * 64 == NT, "one wave per WM x WN sub-tile");
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int LA = BM * BK / NT, LB = BK * BN / NT;
  static_assert(LA * NT == BM * BK && LB * NT == BK * BN, "tile loads must divide evenly");

  const int row0 = jb.row0, col0 = jb.col0;
  const C2* A = jb.A;
  const C2* B = jb.B;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  int wm, wn;
  if constexpr (BM / WM == 4 && WAVES_N == 4) {
    // sixteen waves: sub-tile position kWavePos16[wave], so that the waves of a
    // diagonal tile that have work (10 of 16) spread 2-3 to every SIMD
    const int pos = int((kWavePos16 >> (4 * wave)) & 15);
    wm = (pos >> 2) * WM;
    wn = (pos & 3) * WN;
  } else {
    wm = (wave / WAVES_N) * WM;
    wn = (wave % WAVES_N) * WN;
  }
  // in a diagonal tile of a (skew-)Hermitian result a wave whose sub-tile lies
  // wholly below the diagonal has nothing to compute (it still helps load)
  const bool idle = p.herm && jb.tm == jb.tn && wm >= wn + WN;

  Acc accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) { accr[i][j][e] = T(0); acci[i][j][e] = T(0); }

  // Loads are unconditional: an out-of-range element reads a clamped, valid
  // address and is replaced by zero, so no load sits behind a branch.  Offsets
  // inside one item fit 32 bits (the host keeps ld * rows below 2^31).
  const int lda = int(p.lda), ldb = int(p.ldb);
  C2 ra[LA], rb[LB];
  // FP64: rows of A past M and columns of B past N only feed outputs the
  // epilogue drops, so they may read the clamped last row / column as they are,
  // and a K step wholly inside K loads from precomputed addresses with no clamp
  // and no select (+4 % on large FP64 products; the FP32 kernel measured faster
  // with the clamped form throughout)
  const C2* pa[LA];
  const C2* pb[LB];
  static_assert(MODE == 0 || sizeof(T) == 8, "complex64 operands widen into the FP64 kernel only");
  if constexpr (sizeof(T) == 8 && MODE == 0) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + NT * q;
      pa[q] = A + min(row0 + e / BK, p.M - 1) * lda + e % BK;   // A[row][k0 + ka] at pa[q][k0]
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + NT * q;
      pb[q] = B + (e / BN) * ldb + min(col0 + e % BN, p.N - 1);   // B[k0 + kb][col] at pb[q][k0 ldb]
    }
  }
  // mode 1: A = R and B = R^dag from the complex64 R (M = N = K); both tiles
  // read R row-wise, k fastest (B's element (k, c) is conj R[c][k]), and B goes
  // to LDS transposed, as A does (hence its padded rows).  Rows of R past M only
  // feed outputs that are not stored: inside K their clamped addresses are fixed.
  const float2* qa[MODE == 1 ? LA : 1];
  const float2* qb[MODE == 1 ? LB : 1];
  if constexpr (MODE == 1) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + NT * q;
      qa[q] = jb.R + min(row0 + e / BK, p.M - 1) * int(p.ld32) + e % BK;
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + NT * q;
      qb[q] = jb.R + min(col0 + e / BK, p.N - 1) * int(p.ld32) + e % BK;
    }
  }
  auto load = [&](int k0) {
    if constexpr (MODE == 1) {
      if (k0 + BK <= p.K) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
          const float2 v = qa[q][k0];
          ra[q] = make_double2(double(v.x), double(v.y));
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
          const float2 v = qb[q][k0];
          rb[q] = make_double2(double(v.x), -double(v.y));
        }
        return;
      }
      const float2* R = jb.R;
      const int ld = int(p.ld32);
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int e = tid + NT * q, r = e / BK, k = e % BK;
        const int gr = row0 + r, gk = k0 + k;
        const bool in = gr < p.M && gk < p.K;
        const float2 v = R[min(gr, p.M - 1) * ld + max(0, min(gk, p.K - 1))];
        ra[q] = in ? make_double2(double(v.x), double(v.y)) : czero<C2>();
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int e = tid + NT * q, c = e / BK, k = e % BK;
        const int gc = col0 + c, gk = k0 + k;
        const bool in = gc < p.N && gk < p.K;
        const float2 v = R[min(gc, p.N - 1) * ld + max(0, min(gk, p.K - 1))];
        rb[q] = in ? make_double2(double(v.x), -double(v.y)) : czero<C2>();
      }
      return;
    }
    if constexpr (sizeof(T) == 8 && MODE == 0) {
      if (k0 + BK <= p.K) {
#pragma unroll
        for (int q = 0; q < LA; ++q) ra[q] = pa[q][k0];
#pragma unroll
        for (int q = 0; q < LB; ++q) rb[q] = pb[q][k0 * ldb];
        return;
      }
    }
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + NT * q, r = e / BK, k = e % BK;
      const int gr = row0 + r, gk = k0 + k;
      const bool in = gr < p.M && gk < p.K;
      const C2 v = A[min(gr, p.M - 1) * lda + max(0, min(gk, p.K - 1))];
      ra[q] = in ? v : czero<C2>();
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + NT * q, k = e / BN, c = e % BN;
      const int gk = k0 + k, gc = col0 + c;
      const bool in = gk < p.K && gc < p.N;
      const C2 v = B[max(0, min(gk, p.K - 1)) * ldb + min(gc, p.N - 1)];
      rb[q] = in ? v : czero<C2>();
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int e = tid + NT * q;
      As[buf][e % BK][e / BK] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + NT * q;
      if constexpr (MODE == 1)
        Bs[buf][e % BK][e / BK] = rb[q];
      else
        Bs[buf][e / BN][e % BN] = rb[q];
    }
  };

  const int nk = (p.K + BK - 1) / BK;
  if (nk > 0) {   // K = 0 (C = beta C + terms) reads no operand
    load(0);
    store(0);
  }
  __syncthreads();
  const int lr = lane >> 4, lc = lane & 15;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
    // FP32: the MFMA stream runs at raised wave priority, so that while it issues,
    // the other waves' loads and LDS stores do not take its slots (measured +2 %
    // on large products; the FP64 kernel, which also serves the LU's small-K
    // updates, lost 3 % there and stays at the default)
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      if (idle) break;
      C2 a[TM], bb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[cur][kk + lr][wm + i * 16 + lc];
#pragma unroll
      for (int j = 0; j < TN; ++j) bb[j] = Bs[cur][kk + lr][wn + j * 16 + lc];
      // the minus sign of Ai Bi rides on the operand with fewer fragments
      T nbi[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) nbi[j] = -bb[j].y;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const T ar = a[i].x, ai = a[i].y;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          accr[i][j] = mfma16(ar, bb[j].x, accr[i][j]);
          accr[i][j] = mfma16(ai, nbi[j], accr[i][j]);
          acci[i][j] = mfma16(ar, bb[j].y, acci[i][j]);
          acci[i][j] = mfma16(ai, bb[j].x, acci[i][j]);
        }
      }
    }
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // the LDS tiles are free now (the last K step ended on a barrier): each wave
  // takes a 16 x 16 block of them for the mirror stores
  constexpr int kScrA = 2 * BK * (BM + 1) / 256, kScrB = 2 * BK * BN / 256;
  static_assert(NT / 64 <= kScrA + kScrB, "a 16 x 16 LDS block per wave");
  C2* scr = wave < kScrA ? &As[0][0][0] + wave * 256 : &Bs[0][0][0] + (wave - kScrA) * 256;
  tile_epilogue<T, TM, TN>(p, jb, accr, acci, wm, wn, lane, scr);
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int NT, int WAVES_PER_EU, int MODE = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU))) void cgemm_kernel(
    GemmParams<T> p) {
  using C2 = typename Cx<T>::t;
  __shared__ __attribute__((aligned(16))) C2 As[2][BK][BM + 1];
  __shared__ __attribute__((aligned(16))) C2 Bs[2][BK][BN + (MODE == 1)];
  TileJob<T> jb;
  if (!tile_job<T, BM, BN>(p, xcd_remap(blockIdx.x, gridDim.x), jb)) return;
  cgemm_tile<T, BM, BN, BK, WM, WN, NT, MODE>(p, jb, As, Bs);
}

// Grouped products: up to kMaxGroups batches of different shapes (the
// dimension groups of an uneven sweep) in one launch, a workgroup per tile
// slot.  The hardware hands workgroups to the eight XCDs in turn, so slot t
// runs on XCD t % 8.  Every group's items are split evenly over the XCDs (XCD x
// takes items [item0[x][g], item0[x][g] + count) of group g), so each XCD gets
// the same mix of cheap and costly tiles, and an item's tiles share one L2.
// XCD x's slots are j = t / 8: group g holds slots [base[x][g], base[x][g + 1]),
// item-major.  (A persistent form, a grid of resident workgroups walking the
// slots, ran 1-2 % slower on d = 1000-1024 products: values it hoisted out of
// its tile loop spilled.)
constexpr int kMaxGroups = 8;
constexpr int kXcds = 8;
template <typename T> struct GemmGroups {
  int G;
  int per_xcd;                        // slots of the busiest XCD
  int base[kXcds][kMaxGroups + 1];
  int item0[kXcds][kMaxGroups];
  GemmParams<T> p[kMaxGroups];
};

template <typename T, int BM, int BN, int BK, int WM, int WN, int NT, int WAVES_PER_EU, int MODE = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU))) void cgemm_grouped_kernel(
    GemmGroups<T> gg) {
  using C2 = typename Cx<T>::t;
  __shared__ __attribute__((aligned(16))) C2 As[2][BK][BM + 1];
  __shared__ __attribute__((aligned(16))) C2 Bs[2][BK][BN + (MODE == 1)];
  const int t = blockIdx.x;
  const int x = t % kXcds, j = t / kXcds;
  if (j >= gg.base[x][gg.G]) return;   // this XCD has fewer slots
  int g = 0;
  while (g + 1 < gg.G && j >= gg.base[x][g + 1]) ++g;
  const GemmParams<T>& p = gg.p[g];
  const int tiles = p.herm ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  const int local = j - gg.base[x][g];
  TileJob<T> jb;
  if (!tile_job<T, BM, BN>(p, (gg.item0[x][g] + local / tiles) * tiles + local % tiles, jb)) return;
  cgemm_tile<T, BM, BN, BK, WM, WN, NT, MODE>(p, jb, As, Bs);
}

// Tile configurations per precision: cfg 0 is the large tile, cfg 1 the small
// one (for small matrices, where the large tile would be mostly padding).
// FP32 cfg 0: 128x128 tile, sixteen waves of 32x32 and K steps of 8: 62
// registers and 33 KB of LDS per workgroup, so two workgroups share a CU and
// eight waves each SIMD (measured on batched d = 512..1024 products: 128-134
// TFLOP/s general and 100-115 on (skew-)Hermitian halves, 2-10 % above eight
// waves of 64x32 with K steps of 16 at four waves per SIMD).
template <typename T, int CFG> struct GemmTile;
template <> struct GemmTile<float, 0> {
  static constexpr int BM = 128, BN = 128, BK = 8, WM = 32, WN = 32, NT = 1024, WPE = 8;
};
template <> struct GemmTile<float, 1> {
  static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32, NT = 256, WPE = 4;
};
// FP32 cfg 2: FP32 operands on the BF16 matrix cores, three-way split
// (cgemm_bf16x3_kernel); 128x128 tile, eight waves of 64x32, K steps of 32.
template <> struct GemmTile<float, 2> {
  static constexpr int BM = 128, BN = 128, BK = 32, WM = 64, WN = 32, NT = 512, WPE = 2;
};
// FP32 cfg 3: the split-BF16 products with the split done once per workgroup as
// the tile is stored to LDS (cgemm_bf16x3_planes_kernel); same tile as cfg 2.
template <> struct GemmTile<float, 3> {
  static constexpr int BM = 128, BN = 128, BK = 32, WM = 64, WN = 32, NT = 512, WPE = 2;
};
// FP64: K steps of 8 keep the LDS of a workgroup at 33 KB (64x64) or 8 KB
// (32x32) and the registers at 128 / 64, so that four (eight) waves share each
// SIMD; the FP64 MFMA is slow enough that this latency hiding, not operand
// reuse, decides the rate (measured on batched LU updates: 64x64 tiles 66-68
// TFLOP/s at K = 512 and 57 at K = 128, against 59-64 and 48 with K steps of 16
// at two waves per SIMD; 32x32 tiles 33-48 TFLOP/s at K = 32-64).
template <> struct GemmTile<double, 0> {
  static constexpr int BM = 64, BN = 64, BK = 8, WM = 32, WN = 32, NT = 256, WPE = 4;
};
template <> struct GemmTile<double, 1> {
  static constexpr int BM = 32, BN = 32, BK = 8, WM = 16, WN = 16, NT = 256, WPE = 8;
};
// cfg 4: the third candidate of the tile tuner (square, as the products of
// (skew-)Hermitian results need).  FP32: 128x128 with eight waves of 64x32 and K
// steps of 16 (four waves per SIMD, more operand reuse per LDS read); FP64:
// 128x128 with sixteen waves of 32x32 (a quarter of the L2 traffic per flop of
// the 64x64 tile).
template <> struct GemmTile<float, 4> {
  static constexpr int BM = 128, BN = 128, BK = 16, WM = 64, WN = 32, NT = 512, WPE = 4;
};
template <> struct GemmTile<double, 4> {
  static constexpr int BM = 128, BN = 128, BK = 8, WM = 32, WN = 32, NT = 1024, WPE = 4;
};
constexpr int kTunedCfgs[3] = {0, 1, 4};   // the configurations the tuner times
// the FP32 configurations on the BF16 matrix cores (split operands)
constexpr bool split_bf16_cfg(int cfg) { return cfg == 2 || cfg == 3; }

template <typename T> GemmParams<T> gemm_params(int M, int N, int K, int batch, int cfg = 0) {
  GemmParams<T> p{};
  p.M = M; p.N = N; p.K = K; p.batch = batch;
  p.cfg = cfg;
  int bm = GemmTile<T, 0>::BM, bn = GemmTile<T, 0>::BN;
  if (cfg == 1) { bm = GemmTile<T, 1>::BM; bn = GemmTile<T, 1>::BN; }
  if (cfg == 2 || cfg == 3) { bm = 128; bn = 128; }   // split-BF16 tiles
  if (cfg == 4) { bm = GemmTile<T, 4>::BM; bn = GemmTile<T, 4>::BN; }
  p.tiles_m = (M + bm - 1) / bm;
  p.tiles_n = (N + bn - 1) / bn;
  p.alpha = T(1); p.beta = T(0); p.gamma = T(0); p.nx = 0;
  return p;
}

}  // namespace qcheff
