// Fused [13/13] Pade scaling and squaring for small matrices (d <= 32).
//
// One workgroup of four waves takes one item at a time (grid-stride loop over
// the batch) and keeps everything in LDS: the trace reduction, the FP64 norm
// and scaling exponent,
// the six Pade products on 16x16x4 MFMA (one 16x16 output block per wave), the
// FP64 elimination of the augmented system [V - U | V + U] with partial
// pivoting and its back substitution, the squarings, and (FP32 results of
// skew-Hermitian inputs, on request) one FP64 Newton step towards the nearest
// unitary matrix.  Matrices are stored
// zero-padded to 32 x 32, so every product is exact on the padding.
#pragma once

#include "common.hpp"
#include "lu.hpp"

namespace qcheff {

constexpr int kSmallD = 32;

template <typename T> struct SmallLds {
  using C2 = typename Cx<T>::t;
  // M[0] = A (later R and squarings), M[1..3] = A^2, A^4, A^6, M[4] = W, M[5] = V.
  // The FP64 augmented system (32 x 64 double2 = 32 KB) overlays M[1..].
  union {
    C2 M[6][kSmallD][kSmallD + 1];
    struct {
      C2 keep0[kSmallD][kSmallD + 1];
      double2 aug[kSmallD][2 * kSmallD];
    } s;
  } u;
  double colsum[kSmallD];
  double2 mu;   // trace shift
  int piv;
  int sq;
};

// C = A * Beff (+ sum_i xc[i] X_i + gamma I on the d x d block), where
// Beff = B, or bc[0] B + bc[1] B1 + bc[2] B2 when B1 is given.  All operands are
// 32 x 32 LDS matrices; wave w computes the 16 x 16 output block w.
template <typename T>
__device__ __forceinline__ void small_gemm(typename Cx<T>::t (*C)[kSmallD + 1],
                                           const typename Cx<T>::t (*A)[kSmallD + 1],
                                           const typename Cx<T>::t (*B)[kSmallD + 1],
                                           const typename Cx<T>::t (*B1)[kSmallD + 1],
                                           const typename Cx<T>::t (*B2)[kSmallD + 1], const T* bc,
                                           const typename Cx<T>::t (*const* X)[kSmallD + 1], const T* xc, int nx,
                                           T gamma, int d, typename Cx<T>::acc (&outr), typename Cx<T>::acc (&outi),
                                           bool store) {
  using C2 = typename Cx<T>::t;
  using Acc = typename Cx<T>::acc;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nblk = d > 16 ? 2 : 1;
  const int bm = wave >> 1, bn = wave & 1;
  Acc ar, ai;
#pragma unroll
  for (int e = 0; e < 4; ++e) { ar[e] = T(0); ai[e] = T(0); }
  if (bm < nblk && bn < nblk) {
    const int kend = (d + 3) & ~3;
    const int lr = lane >> 4, lc = lane & 15;
    for (int k = 0; k < kend; k += 4) {
      const C2 a = A[bm * 16 + lc][k + lr];
      C2 b = B[k + lr][bn * 16 + lc];
      if (B1) {
        const C2 b1 = B1[k + lr][bn * 16 + lc], b2 = B2[k + lr][bn * 16 + lc];
        b.x = bc[0] * b.x + bc[1] * b1.x + bc[2] * b2.x;
        b.y = bc[0] * b.y + bc[1] * b1.y + bc[2] * b2.y;
      }
      ar = mfma16(a.x, b.x, ar);
      ar = mfma16(-a.y, b.y, ar);
      ai = mfma16(a.x, b.y, ai);
      ai = mfma16(a.y, b.x, ai);
    }
  }
  outr = ar;
  outi = ai;
  if (!store || bm >= nblk || bn >= nblk) return;
  const int c = bn * 16 + (lane & 15);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = bm * 16 + acc_row<T>(lane, e);
    T vr = ar[e], vi = ai[e];
    for (int x = 0; x < nx; ++x) {
      vr += xc[x] * X[x][r][c].x;
      vi += xc[x] * X[x][r][c].y;
    }
    if (r == c && r < d) vr += gamma;
    C2 o;
    o.x = vr;
    o.y = vi;
    C[r][c] = o;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void expm_small_kernel(const typename Cx<T>::t* __restrict__ omega,
                                                         typename Cx<T>::t* __restrict__ U,
                                                         double2* __restrict__ U64, int* __restrict__ s_out,
                                                         int d, int batch, double theta, int refine) {
  using C2 = typename Cx<T>::t;
  using Acc = typename Cx<T>::acc;
  __shared__ SmallLds<T> L;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  auto& Mx = L.u.M;
  double b[14];
  b[0] = 1.0;
  for (int j = 0; j < 13; ++j) b[j + 1] = b[j] * double(13 - j) / (double(26 - j) * double(j + 1));
  T c[14];
  for (int j = 0; j < 14; ++j) c[j] = T(b[j]);
  const int64_t dd = int64_t(d) * d;

  for (int item = blockIdx.x; item < batch; item += gridDim.x) {
    // load, zero-padded to 32 x 32
    const C2* src = omega + item * dd;
    for (int e = tid; e < kSmallD * kSmallD; e += 256) {
      const int i = e / kSmallD, j = e % kSmallD;
      Mx[0][i][j] = (i < d && j < d) ? src[i * d + j] : czero<C2>();
    }
    __syncthreads();
    // trace reduction, in FP64 only (as in the batched path): exp(Omega) =
    // e^mu exp(Omega - mu I), mu = tr(Omega) / d
    constexpr bool kShift = sizeof(T) == 8;
    if (tid == 0) {
      double re = 0.0, im = 0.0;
      for (int i = 0; i < d; ++i) {
        re += double(Mx[0][i][i].x);
        im += double(Mx[0][i][i].y);
      }
      L.mu = kShift ? make_double2(re / d, im / d) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const double2 mu = L.mu;
    if (tid < d) {
      Mx[0][tid][tid].x = T(double(Mx[0][tid][tid].x) - mu.x);
      Mx[0][tid][tid].y = T(double(Mx[0][tid][tid].y) - mu.y);
    }
    __syncthreads();
    // 1-norm in FP64 and the scaling exponent
    if (tid < kSmallD) {
      double sum = 0.0;
      for (int i = 0; i < d; ++i) {
        const C2 v = Mx[0][i][tid];
        sum += sqrt(double(v.x) * double(v.x) + double(v.y) * double(v.y));
      }
      L.colsum[tid] = sum;
    }
    __syncthreads();
    if (tid == 0) {
      double nrm = 0.0;
      for (int j = 0; j < d; ++j) {
        const double v = L.colsum[j];
        if (v > nrm || v != v) nrm = v;
      }
      int s;
      if (!(nrm <= 1.7976931348623157e308)) {
        s = -1;
        flag_status(STATUS_NONFINITE);
      } else {
        s = 0;
        while (nrm > ldexp(theta, s)) ++s;
      }
      L.sq = s;
      if (s_out) s_out[item] = s;
    }
    __syncthreads();
    const int s = L.sq;
    const double f = (s >= 0) ? ldexp(1.0, -s) : __longlong_as_double(0x7ff8000000000000LL);
    for (int e = tid; e < kSmallD * kSmallD; e += 256) {
      const int i = e / kSmallD, j = e % kSmallD;
      C2 v = Mx[0][i][j];
      v.x = T(double(v.x) * f);
      v.y = T(double(v.y) * f);
      if (i >= d || j >= d) v = czero<C2>();
      Mx[0][i][j] = v;
    }
    __syncthreads();
    Acc tr, ti;
    small_gemm<T>(Mx[1], Mx[0], Mx[0], nullptr, nullptr, nullptr, nullptr, nullptr, 0, T(0), d, tr, ti, true);
    __syncthreads();
    small_gemm<T>(Mx[2], Mx[1], Mx[1], nullptr, nullptr, nullptr, nullptr, nullptr, 0, T(0), d, tr, ti, true);
    __syncthreads();
    small_gemm<T>(Mx[3], Mx[2], Mx[1], nullptr, nullptr, nullptr, nullptr, nullptr, 0, T(0), d, tr, ti, true);
    __syncthreads();
    {
      const C2 (*Xs[3])[kSmallD + 1] = {Mx[3], Mx[2], Mx[1]};
      const T bw[3] = {c[13], c[11], c[9]}, xw[3] = {c[7], c[5], c[3]};
      small_gemm<T>(Mx[4], Mx[3], Mx[3], Mx[2], Mx[1], bw, Xs, xw, 3, c[1], d, tr, ti, true);
      const T bv[3] = {c[12], c[10], c[8]}, xv[3] = {c[6], c[4], c[2]};
      small_gemm<T>(Mx[5], Mx[3], Mx[3], Mx[2], Mx[1], bv, Xs, xv, 3, c[0], d, tr, ti, true);
    }
    __syncthreads();
    // U = A W kept in registers until the augmented system may overwrite M[1..]
    small_gemm<T>(nullptr, Mx[0], Mx[4], nullptr, nullptr, nullptr, nullptr, nullptr, 0, T(0), d, tr, ti, false);
    __syncthreads();
    {
      const int nblk = d > 16 ? 2 : 1, bm = wave >> 1, bn = wave & 1;
      if (bm < nblk && bn < nblk) {
        const int col = bn * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = bm * 16 + acc_row<T>(lane, e);
          const C2 v = Mx[5][r][col];
          const double ur = double(tr[e]), ui = double(ti[e]);
          L.u.s.aug[r][col] = make_double2(double(v.x) - ur, double(v.y) - ui);
          L.u.s.aug[r][kSmallD + col] = make_double2(double(v.x) + ur, double(v.y) + ui);
        }
      }
    }
    __syncthreads();
    // Gaussian elimination with partial pivoting on [q | p]: rows [0, d),
    // columns [0, d) and [32, 32 + d).  Only the reduced system is needed, so
    // the multipliers are formed on the fly and not stored.
    auto& G = L.u.s.aug;
    for (int j = 0; j < d; ++j) {
      if (wave == 0) {
        double v = -1.0;
        int idx = 0x7fffffff;
        if (lane >= j && lane < d) {
          v = pivot_mag(G[lane][j]);
          idx = lane;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(v, off);
          const int oi = __shfl_xor(idx, off);
          argmax_combine(v, idx, ov, oi);
        }
        if (lane == 0) L.piv = (idx >= j && idx < d) ? idx : j;
      }
      __syncthreads();
      const int p = L.piv;
      if (p != j && tid < 2 * kSmallD) {
        const double2 t = G[j][tid];
        G[j][tid] = G[p][tid];
        G[p][tid] = t;
      }
      __syncthreads();
      const double2 inv = crecip(G[j][j]);
      const int rows = d - j - 1, cols = 2 * kSmallD - j - 1;
      for (int e = tid; e < rows * cols; e += 256) {
        const int i = j + 1 + e / cols, cc = j + 1 + e % cols;
        const double2 l = cmul(G[i][j], inv);
        const double2 t = cmul(l, G[j][cc]);
        G[i][cc].x -= t.x;
        G[i][cc].y -= t.y;
      }
      __syncthreads();
    }
    // back substitution, one thread per right-hand-side column
    if (tid < d) {
      const int col = kSmallD + tid;
      for (int i = d - 1; i >= 0; --i) {
        double2 v = G[i][col];
        for (int k = i + 1; k < d; ++k) {
          const double2 t = cmul(G[i][k], G[k][col]);
          v.x -= t.x;
          v.y -= t.y;
        }
        G[i][col] = cmul(v, crecip(G[i][i]));
      }
    }
    __syncthreads();
    // R into M[0] (rounded to T), zero-padded; the squarings ping-pong with M[5]
    for (int e = tid; e < kSmallD * kSmallD; e += 256) {
      const int i = e / kSmallD, j = e % kSmallD;
      C2 v = czero<C2>();
      if (i < d && j < d) {
        const double2 r = G[i][kSmallD + j];
        v.x = T(r.x);
        v.y = T(r.y);
      }
      Mx[0][i][j] = v;
    }
    __syncthreads();
    int cur = 0;
    for (int k = 0; k < s; ++k) {
      const int nxt = cur == 0 ? 5 : 0;
      small_gemm<T>(Mx[nxt], Mx[cur], Mx[cur], nullptr, nullptr, nullptr, nullptr, nullptr, 0, T(0), d, tr, ti,
                    true);
      __syncthreads();
      cur = nxt;
    }
    if (refine) {
      // One Newton step of the polar decomposition in FP64 (the FP32 squarings
      // leave |eigenvalues| off 1 by about 2^s u32): E = I - R R^dag, then
      // R' = R + (1/2) E R.  E takes the space of the augmented system.
      auto& E = L.u.s.aug;
      for (int e = tid; e < d * d; e += 256) {
        const int i = e / d, j = e % d;
        double gr = 0.0, gi = 0.0;
        for (int k = 0; k < d; ++k) {
          const C2 a = Mx[cur][i][k], b = Mx[cur][j][k];   // a conj(b)
          gr += double(a.x) * double(b.x) + double(a.y) * double(b.y);
          gi += double(a.y) * double(b.x) - double(a.x) * double(b.y);
        }
        E[i][j] = make_double2((i == j ? 1.0 : 0.0) - gr, -gi);
      }
      __syncthreads();
      for (int e = tid; e < d * d; e += 256) {
        const int i = e / d, j = e % d;
        double cr = 0.0, ci = 0.0;
        for (int k = 0; k < d; ++k) {
          const double2 a = E[i][k];
          const C2 b = Mx[cur][k][j];
          cr += a.x * double(b.x) - a.y * double(b.y);
          ci += a.x * double(b.y) + a.y * double(b.x);
        }
        const C2 v = Mx[cur][i][j];
        const double2 r = make_double2(double(v.x) + 0.5 * cr, double(v.y) + 0.5 * ci);
        if (U64) {   // kept in FP64
          U64[item * dd + e] = r;
        } else {
          C2 o;
          o.x = T(r.x);
          o.y = T(r.y);
          U[item * dd + e] = o;
        }
      }
    } else {
      C2* dst = U + item * dd;
      const double er = exp(mu.x), pr = er * cos(mu.y), pi = er * sin(mu.y);
      for (int e = tid; e < d * d; e += 256) {
        const C2 v = Mx[cur][e / d][e % d];
        C2 o;
        o.x = T(pr * double(v.x) - pi * double(v.y));
        o.y = T(pr * double(v.y) + pi * double(v.x));
        dst[e] = o;
      }
    }
    __syncthreads();
  }
}

}  // namespace qcheff
