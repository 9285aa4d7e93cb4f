// Device kernels of the Magnus path other than the GEMM (gfx950).
#pragma once

#include "common.hpp"

namespace qcheff {

// ---------------------------------------------------------------- helpers

// Neumaier's compensated summation (Neumaier 1974): running sum plus a
// correction term that collects the rounding error of every addition.
struct Neumaier {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

template <typename C2> __device__ __forceinline__ C2 to_c2(double re, double im);
template <> __device__ __forceinline__ float2 to_c2<float2>(double re, double im) {
  return make_float2(float(re), float(im));
}
template <> __device__ __forceinline__ double2 to_c2<double2>(double re, double im) {
  return make_double2(re, im);
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------ coefficients
//
// One wave per interval n.  The interval's s samples are taken in rounds of 64
// consecutive samples, one per lane, so every load of a round is one coalesced
// 512-byte read.
//   c1[n][k]    = dt * sum_j u_k[j]
//   c2[n][k]    = dt^2 * sum_j (s - 1 - 2j) u_k[j]
//   c2[n][K+p]  = dt^2 * sum_j (u_k[j] P_l[j] - u_l[j] P_k[j]),  P[j] = sum_{i<j} u[i]
// Each lane keeps compensated (Neumaier) sums of its samples; the 64 partial
// sums are combined by a fixed tree of error-free additions (Knuth's two-sum),
// so the result does not depend on timing.  The prefix sums P come from a scan
// across the lanes of each round plus the running total of earlier rounds.

// s + e = a + b exactly, s = fl(a + b) (Knuth's two-sum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Sum over the wave of the lanes' (sum, compensation) pairs; valid in lane 0.
__device__ __forceinline__ double wave_sum_compensated(double s, double c) {
  for (int off = 32; off > 0; off >>= 1) {
    const double so = __shfl_down(s, off), co = __shfl_down(c, off);
    double t, e;
    two_sum(s, so, t, e);
    s = t;
    c += co + e;
  }
  return s + c;
}

// Inclusive prefix sum of x over the lanes of a wave.
__device__ __forceinline__ double wave_inclusive_scan(double x, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

__global__ __launch_bounds__(256) void coeffs_kernel(const double* __restrict__ u, int K, int64_t N, int64_t M,
                                                     int64_t s, double dt, int order, double* __restrict__ c1,
                                                     double* __restrict__ c2, int ldc2) {
  const int lane = threadIdx.x & 63;
  const int64_t n = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (n >= M) return;   // a whole wave leaves together
  const int64_t base = n * s;
  const int P2 = ldc2;   // row stride of c2 (the second-order columns come first)
  for (int k = 0; k < K; ++k) {
    const double* uk = u + int64_t(k) * N + base;
    Neumaier sum, wsum;
    for (int64_t j = lane; j < s; j += 64) {
      const double x = uk[j];
      sum.add(x);
      if (order >= 2) wsum.add(double(s - 1 - 2 * j) * x);
    }
    const double c1v = wave_sum_compensated(sum.s, sum.c);
    const double c20 = wave_sum_compensated(wsum.s, wsum.c);
    if (lane == 0) {
      c1[n * K + k] = dt * c1v;
      if (order >= 2) c2[n * P2 + k] = dt * dt * c20;
    }
  }
  if (order < 2) return;
  int p = K;
  for (int k = 0; k < K; ++k) {
    for (int l = k + 1; l < K; ++l, ++p) {
      const double* uk = u + int64_t(k) * N + base;
      const double* ul = u + int64_t(l) * N + base;
      Neumaier acc;
      double carry_k = 0.0, carry_l = 0.0;   // sums of the earlier rounds
      for (int64_t j0 = 0; j0 < s; j0 += 64) {
        const int64_t j = j0 + lane;
        const double xk = j < s ? uk[j] : 0.0, xl = j < s ? ul[j] : 0.0;
        const double ik = wave_inclusive_scan(xk, lane), il = wave_inclusive_scan(xl, lane);
        const double pk = carry_k + (ik - xk), pl = carry_l + (il - xl);   // exclusive prefixes
        acc.add(xk * pl);
        acc.add(-(xl * pk));
        carry_k += __shfl(ik, 63);
        carry_l += __shfl(il, 63);
      }
      const double v = wave_sum_compensated(acc.s, acc.c);
      if (lane == 0) c2[n * P2 + p] = dt * dt * v;
    }
  }
}

// Third-order coefficients: for the index triples q = (a, b, c) of {0..K}^3 with
// a <= c and not a = b = c (in the order a, then c, then b; x_0 = 1 is the drift,
// x_k = u_{k-1}), c2[n][col0 + q] = T_abc + T_cba (a < c) or T_aba (a = c), where
// T_abc = int_{t3<t2<t1} x_a(t1) x_b(t2) x_c(t3) over interval n.  For a
// zero-order-hold signal, cells i > j > k add dt^3 x_a[i] x_b[j] x_c[k], ties add
// half (i = j or j = k) or a sixth (all equal) of that; with running sums
// C = sum_{k<j} x_c[k], Q = sum_{j<i} x_b[j] C[j], R = sum_{j<i} x_b[j] x_c[j] each
// cell i adds x_a[i] (Q + x_b[i] C / 2 + R / 2 + x_b[i] x_c[i] / 6).  One wave per
// interval, one lane per triple walking the samples in time order; the samples
// pass through LDS in tiles of 256 per control, loaded by the whole wave.
constexpr int kC3Tile = 256;

__device__ __forceinline__ bool c3_triple(int q, int K, int& a, int& b, int& c) {
  int r = 0;
  for (a = 0; a <= K; ++a)
    for (c = a; c <= K; ++c)
      for (b = 0; b <= K; ++b) {
        if (a == b && b == c) continue;
        if (r++ == q) return true;
      }
  return false;
}

__global__ __launch_bounds__(256) void coeffs3_kernel(const double* __restrict__ u, int K, int64_t N, int64_t M,
                                                      int64_t s, double dt, int ldc2, int col0,
                                                      double* __restrict__ c2) {
  __shared__ double tile[4][3][kC3Tile];   // per wave, K <= 3 controls
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n = int64_t(blockIdx.x) * 4 + wave;
  int a = 0, b = 0, c = 0;
  const bool mine = n < M && c3_triple(lane, K, a, b, c);
  double C1 = 0.0, Q1 = 0.0, R1 = 0.0, C2 = 0.0, Q2 = 0.0, R2 = 0.0;
  Neumaier T1, T2;
  for (int64_t t0 = 0; t0 < s; t0 += kC3Tile) {   // the same trip count in every wave
    const int cnt = int(min(int64_t(kC3Tile), s - t0));
    if (n < M)
      for (int k = 0; k < K; ++k)
        for (int l = lane; l < cnt; l += 64) tile[wave][k][l] = u[int64_t(k) * N + n * s + t0 + l];
    __syncthreads();
    if (mine) {
      for (int i = 0; i < cnt; ++i) {
        const double xa = a ? tile[wave][a - 1][i] : 1.0;
        const double xb = b ? tile[wave][b - 1][i] : 1.0;
        const double xc = c ? tile[wave][c - 1][i] : 1.0;
        T1.add(xa * (Q1 + 0.5 * xb * C1 + 0.5 * R1 + xb * xc * (1.0 / 6.0)));
        Q1 += xb * C1;
        R1 += xb * xc;
        C1 += xc;
        T2.add(xc * (Q2 + 0.5 * xb * C2 + 0.5 * R2 + xb * xa * (1.0 / 6.0)));
        Q2 += xb * C2;
        R2 += xb * xa;
        C2 += xa;
      }
    }
    __syncthreads();
  }
  if (mine) {
    const double v = a < c ? T1.value() + T2.value() : T1.value();
    c2[n * ldc2 + col0 + lane] = dt * dt * dt * v;
  }
}

// C = (X1 + X1^dag) + (X2 + X2^dag) for square d x d matrices (X1 or X2 null: left
// out): the third-order basis element [H_a, D1] + [H_c, D2] from X1 = H_a D1,
// X2 = H_c D2 with Hermitian H and anti-Hermitian D (then [H, D] = H D + (H D)^dag).
__global__ void hermitian_sum_kernel(const double2* __restrict__ X1, const double2* __restrict__ X2,
                                     double2* __restrict__ C, int d) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(d) * d) return;
  const int64_t i = e / d, j = e % d;
  const int64_t t = j * d + i;
  double re = 0.0, im = 0.0;
  if (X1) {
    re += X1[e].x + X1[t].x;
    im += X1[e].y - X1[t].y;
  }
  if (X2) {
    re += X2[e].x + X2[t].x;
    im += X2[e].y - X2[t].y;
  }
  C[e] = make_double2(re, im);
}

// ------------------------------------------------------ commutator basis
//
// In place: C <- X - X^dag for a square d x d matrix (X = F G for Hermitian F,
// G gives [F, G] = F G - (F G)^dag, exactly anti-Hermitian).
__global__ void antihermitian_part_kernel(double2* X, int d) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(d) * d) return;
  const int i = int(e / d), j = int(e % d);
  if (i > j) return;
  const double2 a = X[int64_t(i) * d + j];
  if (i == j) {
    X[e] = make_double2(0.0, 2.0 * a.y);
    return;
  }
  const double2 b = X[int64_t(j) * d + i];
  const double2 cij = make_double2(a.x - b.x, a.y + b.y);  // a - conj(b)
  X[int64_t(i) * d + j] = cij;
  X[int64_t(j) * d + i] = make_double2(-cij.x, cij.y);     // -conj(cij)
}

// ------------------------------------------------------------- generators
//
// Omega_n[e] = -i ( dt H0[e] + sum_k c1[n][k] H_k[e] - (i/2) sum_p c2[n][p] C_p[e]
//                  - (1/6) sum_q c3[n][q] C3_q[e] )   (the last term at order 3)
// One thread per matrix element e holds the operator values in registers and
// walks a chunk of intervals; coefficients of the chunk sit in LDS.
template <int K, int ORDER, typename OutC2>
__global__ __launch_bounds__(256) void generators_kernel(const double2* __restrict__ H0,
                                                         const double2* __restrict__ Hk,
                                                         const double2* __restrict__ Cb, int64_t dd,
                                                         const double* __restrict__ c1,
                                                         const double* __restrict__ c2, int64_t M,
                                                         int nch, double dt, OutC2* __restrict__ omega) {
  constexpr int P2 = (ORDER >= 2) ? K + K * (K - 1) / 2 : 0;
  constexpr int P3 = (ORDER == 3) ? (K + 1) * K * (K + 3) / 2 : 0;
  constexpr int NC = K + P2 + P3;
  extern __shared__ double sh[];  // [nch][NC]
  const int64_t n0 = int64_t(blockIdx.y) * nch;
  const int cnt = int(min(int64_t(nch), M - n0));
  for (int i = threadIdx.x; i < cnt * NC; i += blockDim.x) {
    const int r = i / NC, q = i % NC;
    sh[i] = (q < K) ? c1[(n0 + r) * K + q] : c2[(n0 + r) * (P2 + P3) + (q - K)];
  }
  __syncthreads();
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= dd) return;
  const double2 h0 = H0[e];
  double2 hk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) hk[k] = Hk[int64_t(k) * dd + e];
  double2 cb[P2 + P3 > 0 ? P2 + P3 : 1];   // second-order basis, then the third-order one
#pragma unroll
  for (int q = 0; q < P2 + P3; ++q) cb[q] = Cb[int64_t(q) * dd + e];
  for (int r = 0; r < cnt; ++r) {
    const double* cf = sh + r * NC;
    double hr = dt * h0.x, hi = dt * h0.y;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      hr += cf[k] * hk[k].x;
      hi += cf[k] * hk[k].y;
    }
    if constexpr (ORDER >= 2) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < P2; ++q) {
        sr += cf[K + q] * cb[q].x;
        si += cf[K + q] * cb[q].y;
      }
      hr += 0.5 * si;   // -(i/2) (sr + i si) = si/2 - i sr/2
      hi -= 0.5 * sr;
    }
    if constexpr (ORDER == 3) {
      // -(1/6) sum_q c3[q] ([H_a,[H_b,H_c]] + [H_c,[H_b,H_a]])
      double tr = 0.0, ti = 0.0;
#pragma unroll
      for (int q = 0; q < P3; ++q) {
        tr += cf[K + P2 + q] * cb[P2 + q].x;
        ti += cf[K + P2 + q] * cb[P2 + q].y;
      }
      hr -= tr * (1.0 / 6.0);
      hi -= ti * (1.0 / 6.0);
    }
    omega[(n0 + r) * dd + e] = to_c2<OutC2>(hi, -hr);  // -i (hr + i hi)
  }
}

// ------------------------------------------------------ norm and scaling
//
// Column sums of |Omega - mu I| in FP64 in two launches.  The first reads a
// 64-column by 128-row tile per workgroup (each wave one row at a time, so a
// wave's load is 64 consecutive elements of a row; eight rows in flight per
// lane) and writes the tile's partial column sums; the second adds the row
// tiles' partials of each column in a fixed order and takes the largest column
// sum (a NaN wins), so the result is deterministic.
constexpr int kNormRows = 128;   // rows per partial sum

template <typename C2>
__global__ __launch_bounds__(256) void norm1_partial_kernel(const C2* __restrict__ X, int d,
                                                            const double2* __restrict__ mu,
                                                            double* __restrict__ partial) {
  const int b = blockIdx.z, rt = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = blockIdx.x * 64 + lane;
  const int r0 = rt * kNormRows;
  const int r1 = min(d, r0 + kNormRows);
  const double2 m = mu ? mu[b] : make_double2(0.0, 0.0);   // the norm is of X - mu I
  const C2* Xb = X + int64_t(b) * d * d;
  const int cc = min(col, d - 1);
  double sum = 0.0;
  for (int i0 = r0 + wave; i0 < r1; i0 += 4 * 8) {
    C2 v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = i0 + 4 * t;
      v[t] = Xb[int64_t(min(i, d - 1)) * d + cc];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = i0 + 4 * t;
      if (i < r1) {
        double x = double(v[t].x), y = double(v[t].y);
        if (i == col) {
          x -= m.x;
          y -= m.y;
        }
        sum += sqrt(x * x + y * y);
      }
    }
  }
  __shared__ double red[4][64];
  red[wave][lane] = sum;
  __syncthreads();
  if (wave == 0 && col < d) {
    const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    partial[(int64_t(b) * gridDim.y + rt) * d + col] = t;
  }
}

__global__ __launch_bounds__(256) void norm1_finish_kernel(const double* __restrict__ partial, int d, int tiles,
                                                           unsigned long long* __restrict__ norms) {
  const int b = blockIdx.x;
  const double* pb = partial + int64_t(b) * tiles * d;
  double best = 0.0;
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double c = 0.0;
    for (int t = 0; t < tiles; ++t) c += pb[int64_t(t) * d + j];
    if (c > best || c != c) best = c;   // a comparison with NaN is false: test it explicitly
  }
  __shared__ double red[256];
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = red[threadIdx.x + w];
      if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[b] = (unsigned long long)__double_as_longlong(red[0]);
}

// s = smallest s >= 0 with nrm <= theta * 2^s (exact comparisons); -1 if nrm is not finite.
__device__ __forceinline__ int squarings_for(double nrm, double theta) {
  if (!(nrm <= 1.7976931348623157e308)) return -1;
  int s = 0;
  while (nrm > ldexp(theta, s)) ++s;
  return s;
}

// A = (Omega - mu I) / 2^s per item (the shift in FP64, the scaling exact);
// records s.  With bound >= 0 an item whose s exceeds it is recorded as -2 and
// scaled by NaN (its result is all NaN).  mu may be null (no shift).
template <typename C2>
__global__ __launch_bounds__(256) void scale_kernel(const C2* __restrict__ omega, C2* __restrict__ A, int d,
                                                    const double2* __restrict__ mu,
                                                    const unsigned long long* __restrict__ norms, double theta,
                                                    int bound, int* __restrict__ s_ws, int* __restrict__ s_out,
                                                    int* __restrict__ smax) {
  using T = decltype(C2().x);
  const int b = blockIdx.y;
  const int64_t dd = int64_t(d) * d;
  const double nrm = __longlong_as_double((long long)norms[b]);
  const double2 m = mu ? mu[b] : make_double2(0.0, 0.0);
  int s = squarings_for(nrm, theta);
  if (bound >= 0 && s > bound) s = -2;   // needs more squarings than enqueued: NaN result
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s_ws[b] = s;
    if (s_out) s_out[b] = s;
    atomicMax(smax, s);
    if (s == -1) flag_status(STATUS_NONFINITE);
  }
  const double f = (s >= 0) ? ldexp(1.0, -s) : __longlong_as_double(0x7ff8000000000000LL);
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < dd; e += int64_t(gridDim.x) * blockDim.x) {
    const C2 v = omega[b * dd + e];
    C2 o;
    if (e % (d + 1) == 0) {   // diagonal
      o.x = T((double(v.x) - m.x) * f);
      o.y = T((double(v.y) - m.y) * f);
    } else {
      o.x = v.x * T(f);
      o.y = v.y * T(f);
    }
    A[b * dd + e] = o;
  }
}

// U_b <- e^{mu_b} U_b: the factor the trace reduction split off.
template <typename C2>
__global__ __launch_bounds__(256) void phase_kernel(C2* __restrict__ U, int64_t dd, const double2* __restrict__ mu) {
  using T = decltype(C2().x);
  const int b = blockIdx.y;
  const double2 m = mu[b];
  const double er = exp(m.x), pr = er * cos(m.y), pi = er * sin(m.y);
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < dd; e += int64_t(gridDim.x) * blockDim.x) {
    const C2 v = U[b * dd + e];
    C2 o;
    o.x = T(pr * double(v.x) - pi * double(v.y));
    o.y = T(pr * double(v.y) + pi * double(v.x));
    U[b * dd + e] = o;
  }
}

// The inner Pade combinations of both polynomials in one elementwise pass:
// P = w0 A6 + w1 A4 + w2 A2 and Q = v0 A6 + v1 A4 + v2 A2 (the right operands
// of the W and V products), over n elements of the chunk.
template <typename C2, typename T>
__global__ __launch_bounds__(256) void pade_inner_kernel(const C2* __restrict__ A6, const C2* __restrict__ A4,
                                                         const C2* __restrict__ A2, int64_t n, T w0, T w1, T w2,
                                                         T v0, T v1, T v2, C2* __restrict__ P, C2* __restrict__ Q) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const C2 a6 = A6[e], a4 = A4[e], a2 = A2[e];
    C2 pv, qv;
    pv.x = w0 * a6.x + w1 * a4.x + w2 * a2.x;
    pv.y = w0 * a6.y + w1 * a4.y + w2 * a2.y;
    qv.x = v0 * a6.x + v1 * a4.x + v2 * a2.x;
    qv.y = v0 * a6.y + v1 * a4.y + v2 * a2.y;
    P[e] = pv;
    Q[e] = qv;
  }
}

// ------------------------------------------------------ unitary refinement
//
// The FP32 squarings double the deviation of every |eigenvalue| of R from 1 at
// each step, so after s of them the propagator is off unitarity by about
// 2^s u32.  One Newton step of the polar decomposition removes that radial
// error: with E = I - U U^dag (formed in FP64 from the FP32 values),
// U' = U + (1/2) E U is unitary up to O(|E|^2).  Both steps are GEMMs: the
// FP64 kernel reads U's complex64 values itself and writes E in complex64, and
// the FP32 kernel adds (1/2) E U to U in FP64 (cgemm.hpp, EPI_C32, EPI_OUT64).

// ---------------------------------------------------------------- chain
//
// y = U x with U in C2 (FP32 or FP64) and x, y in FP64.  Vec16: the 16-byte
// piece of a row (two complex64 values or one complex128).
template <typename C2> struct Vec16;
template <> struct Vec16<float2> { using t = float4; static constexpr int per = 2; };
template <> struct Vec16<double2> { using t = double2; static constexpr int per = 1; };

// y = U x with a workgroup of NT threads per row: thread t takes the row's
// 16-byte pieces t, t + NT, ... (eight in flight per round, U read with
// nontemporal loads: each element is used once) with the matching entries of x
// (from L2), and the workgroup sums its waves' parts in LDS.  With about eight
// pieces per thread (NT = 128 at d = 1024 in complex128) the chip holds a few
// waves per SIMD instead of the one a wave per row leaves it (complex128 at
// d = 1024: 5.0 against 6.6 us per product).  Rows must be 16-byte aligned:
// complex128, or complex64 with an even d.
template <typename C2> struct Nt16;
template <> struct Nt16<float2> { typedef float t __attribute__((ext_vector_type(4))); };
template <> struct Nt16<double2> { typedef double t __attribute__((ext_vector_type(2))); };

template <typename C2, int NT>
__global__ __launch_bounds__(NT) void matvec_rows_kernel(const C2* __restrict__ U, const double2* __restrict__ x,
                                                         double2* __restrict__ y, int d) {
  using V = typename Nt16<C2>::t;
  using T = decltype(C2().x);
  constexpr int PER = Vec16<C2>::per, MAXP = 8;
  const int row = blockIdx.x;
  const V* ur = reinterpret_cast<const V*>(U + int64_t(row) * d);
  const int nch = d / PER;
  double ar = 0.0, ai = 0.0;
  for (int base = 0; base < nch; base += NT * MAXP) {
    V ub[MAXP];
    double2 xb[MAXP][PER];
#pragma unroll
    for (int t = 0; t < MAXP; ++t) {
      const int c = base + int(threadIdx.x) + NT * t;
      const int cc = c < nch ? c : 0;
      ub[t] = __builtin_nontemporal_load(ur + cc);
#pragma unroll
      for (int q = 0; q < PER; ++q) xb[t][q] = x[cc * PER + q];
    }
#pragma unroll
    for (int t = 0; t < MAXP; ++t) {
      const int c = base + int(threadIdx.x) + NT * t;
      if (c < nch) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const double ur_ = double(T(ub[t][2 * q])), ui_ = double(T(ub[t][2 * q + 1]));
          ar += ur_ * xb[t][q].x - ui_ * xb[t][q].y;
          ai += ur_ * xb[t][q].y + ui_ * xb[t][q].x;
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_down(ar, off);
    ai += __shfl_down(ai, off);
  }
  __shared__ double2 part[NT / 64];
  const int wave = int(threadIdx.x) >> 6, lane = int(threadIdx.x) & 63;
  if (lane == 0) part[wave] = make_double2(ar, ai);
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 sum = part[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) {
      sum.x += part[w].x;
      sum.y += part[w].y;
    }
    y[row] = sum;
  }
}

// Any d: one 8- or 16-byte element per lane per step.
template <typename C2>
__global__ __launch_bounds__(256) void matvec_kernel(const C2* __restrict__ U, const double2* __restrict__ x,
                                                     double2* __restrict__ y, int d) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= d) return;
  const C2* ur = U + int64_t(row) * d;
  double ar = 0.0, ai = 0.0;
  for (int c = lane; c < d; c += 64) {
    const C2 u = ur[c];
    const double2 v = x[c];
    ar += double(u.x) * v.x - double(u.y) * v.y;
    ai += double(u.x) * v.y + double(u.y) * v.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_down(ar, off);
    ai += __shfl_down(ai, off);
  }
  if (lane == 0) y[row] = make_double2(ar, ai);
}

// B independent state chains at once: chain b runs psi <- U[b][n] psi for
// n = 0..M-1 inside one workgroup (one wave per row at a time, the state in
// LDS in FP64), so a single launch covers every chain and every interval.
template <typename C2>
__global__ __launch_bounds__(256) void chain_batched_kernel(const C2* __restrict__ U, double2* __restrict__ x,
                                                            int M, int d) {
  extern __shared__ double2 sv[];   // [2][d]
  const int b = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t dd = int64_t(d) * d;
  double2* xb = x + int64_t(b) * d;
  double2* cur = sv;
  double2* nxt = sv + d;
  for (int i = threadIdx.x; i < d; i += 256) cur[i] = xb[i];
  __syncthreads();
  const C2* Ub = U + int64_t(b) * M * dd;
  for (int n = 0; n < M; ++n) {
    const C2* Un = Ub + n * dd;
    for (int row = wave; row < d; row += 4) {
      const C2* ur = Un + int64_t(row) * d;
      double ar = 0.0, ai = 0.0;
      for (int c = lane; c < d; c += 64) {
        const C2 u = ur[c];
        const double2 v = cur[c];
        ar += double(u.x) * v.x - double(u.y) * v.y;
        ai += double(u.x) * v.y + double(u.y) * v.x;
      }
      for (int off = 32; off > 0; off >>= 1) {
        ar += __shfl_down(ar, off);
        ai += __shfl_down(ai, off);
      }
      if (lane == 0) nxt[row] = make_double2(ar, ai);
    }
    __syncthreads();
    double2* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (int i = threadIdx.x; i < d; i += 256) xb[i] = cur[i];
}

}  // namespace qcheff
