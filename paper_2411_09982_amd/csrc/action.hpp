// State-only propagation: psi <- exp(Omega) psi by a truncated Taylor series of
// the action, never forming exp(Omega) (O(d^2) per matrix-vector product instead
// of O(d^3) per propagator).
//
// Per interval: mu = tr(Omega) / d shifts the generator (exp(Omega) =
// e^mu exp(Omega - mu I); for the Magnus generators of a drift-dominated system
// this removes the large mean diagonal), nu bounds ||Omega - mu I||_2 by
// sqrt(||.||_1 ||.||_inf), and the host picks the Taylor degree m and the number
// of steps s that minimise m s subject to s * sum_{k>m} (nu/s)^k / k! <= tol.
// Then s times: F = b; b <- (Omega - mu I) b / (s j), F += b for j = 1..m;
// b = F = e^{mu/s} F.  Every product reads Omega once (HBM-bound) and
// accumulates in FP64; the state stays in FP64.
#pragma once

#include "common.hpp"

namespace qcheff {

// mu[b] = tr(Omega_b) / d in FP64 (one workgroup per item).
template <typename C2>
__global__ __launch_bounds__(256) void trace_mean_kernel(const C2* __restrict__ X, int d, double2* __restrict__ mu) {
  const int b = blockIdx.x;
  const C2* A = X + int64_t(b) * d * d;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    const C2 v = A[int64_t(i) * d + i];
    re += double(v.x);
    im += double(v.y);
  }
  __shared__ double rr[256], ri[256];
  rr[threadIdx.x] = re;
  ri[threadIdx.x] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rr[threadIdx.x] += rr[threadIdx.x + w];
      ri[threadIdx.x] += ri[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) mu[b] = make_double2(rr[0] / d, ri[0] / d);
}

__device__ __forceinline__ double shifted_abs(double x, double y, bool diag, double2 mu) {
  if (diag) {
    x -= mu.x;
    y -= mu.y;
  }
  return sqrt(x * x + y * y);
}

__device__ __forceinline__ void nan_max(double& a, double o) {
  if (o > a || o != o) a = o;   // NaN wins
}

// norms[2 b] = max column sum, norms[2 b + 1] = max row sum of |Omega_b - mu_b I|,
// as IEEE bits under an atomic max (monotone for non-negative values, NaN the
// largest pattern).  Grid (ceil(d / 256), batch, 2): z = 0 columns, z = 1 rows
// (a wave per row, so that the reads are coalesced).
template <typename C2>
__global__ __launch_bounds__(256) void shifted_norms_kernel(const C2* __restrict__ X, int d,
                                                            const double2* __restrict__ mu,
                                                            unsigned long long* __restrict__ norms) {
  const int b = blockIdx.y;
  const C2* A = X + int64_t(b) * d * d;
  const double2 m = mu[b];
  double best = 0.0;
  if (blockIdx.z == 0) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < d) {
      double sum = 0.0;
      for (int i = 0; i < d; ++i) {
        const C2 v = A[int64_t(i) * d + j];
        sum += shifted_abs(double(v.x), double(v.y), i == j, m);
      }
      best = sum;
    }
  } else {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // rows blockIdx.x * 256 + wave, + 4, ...: 64 rows per wave
    for (int r = blockIdx.x * 256 + wave; r < min(d, int(blockIdx.x) * 256 + 256); r += 4) {
      double sum = 0.0;
      for (int c = lane; c < d; c += 64) {
        const C2 v = A[int64_t(r) * d + c];
        sum += shifted_abs(double(v.x), double(v.y), r == c, m);
      }
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      nan_max(best, sum);
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) nan_max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(norms + 2 * b + blockIdx.z, (unsigned long long)__double_as_longlong(red[0]));
}

// One Taylor term: y = coef (A - mu I) x, F += y; on the last term of a step
// F <- eta F and y <- F (the next step starts from the new F).  A wave per row,
// four independent loads in flight per lane.
template <typename C2>
__global__ __launch_bounds__(256) void action_term_kernel(const C2* __restrict__ A, int d,
                                                          const double2* __restrict__ x, double2* __restrict__ y,
                                                          double2* __restrict__ F, double coef, double2 mu, int last,
                                                          double2 eta) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= d) return;
  const C2* ar = A + int64_t(row) * d;
  double sr = 0.0, si = 0.0;
  int c = lane;
  if constexpr (sizeof(C2) == 8) {
    if ((d & 1) == 0) {
      // complex64 rows of even length start on 16 bytes: a lane reads two
      // elements per load, 1 KB per wave-wide load
      const float4* a4 = reinterpret_cast<const float4*>(ar);
      int c2 = lane;   // index of an element pair
      const int np = d / 2;
      for (; c2 + 192 < np; c2 += 256) {
        float4 u[4];
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          u[q] = a4[c2 + 64 * q];
          v[2 * q] = x[2 * (c2 + 64 * q)];
          v[2 * q + 1] = x[2 * (c2 + 64 * q) + 1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          sr += double(u[q].x) * v[2 * q].x - double(u[q].y) * v[2 * q].y;
          si += double(u[q].x) * v[2 * q].y + double(u[q].y) * v[2 * q].x;
          sr += double(u[q].z) * v[2 * q + 1].x - double(u[q].w) * v[2 * q + 1].y;
          si += double(u[q].z) * v[2 * q + 1].y + double(u[q].w) * v[2 * q + 1].x;
        }
      }
      for (; c2 < np; c2 += 64) {
        const float4 u = a4[c2];
        const double2 v0 = x[2 * c2], v1 = x[2 * c2 + 1];
        sr += double(u.x) * v0.x - double(u.y) * v0.y;
        si += double(u.x) * v0.y + double(u.y) * v0.x;
        sr += double(u.z) * v1.x - double(u.w) * v1.y;
        si += double(u.z) * v1.y + double(u.w) * v1.x;
      }
      c = d;   // the element loop below has nothing left
    }
  }
  for (; c + 192 < d; c += 256) {
    C2 u[4];
    double2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u[q] = ar[c + 64 * q];
      v[q] = x[c + 64 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sr += double(u[q].x) * v[q].x - double(u[q].y) * v[q].y;
      si += double(u[q].x) * v[q].y + double(u[q].y) * v[q].x;
    }
  }
  for (; c < d; c += 64) {
    const C2 u = ar[c];
    const double2 v = x[c];
    sr += double(u.x) * v.x - double(u.y) * v.y;
    si += double(u.x) * v.y + double(u.y) * v.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_down(sr, off);
    si += __shfl_down(si, off);
  }
  if (lane == 0) {
    const double2 xr = x[row];
    sr -= mu.x * xr.x - mu.y * xr.y;
    si -= mu.x * xr.y + mu.y * xr.x;
    const double2 t = make_double2(coef * sr, coef * si);
    double2 f = F[row];
    f.x += t.x;
    f.y += t.y;
    if (last) {
      f = make_double2(eta.x * f.x - eta.y * f.y, eta.x * f.y + eta.y * f.x);
      y[row] = f;
    } else {
      y[row] = t;
    }
    F[row] = f;
  }
}

// x <- eta x (a step with no Taylor term: Omega = mu I exactly, or a
// non-finite generator, eta = NaN).
__global__ __launch_bounds__(256) void scale_state_kernel(double2* __restrict__ x, int d, double2 eta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d) {
    const double2 v = x[i];
    x[i] = make_double2(eta.x * v.x - eta.y * v.y, eta.x * v.y + eta.y * v.x);
  }
}

}  // namespace qcheff
