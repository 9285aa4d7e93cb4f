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

// norms[2 b] = max column sum, norms[2 b + 1] = max row sum of |Omega_b - mu_b I|
// for b = b0 + blockIdx.y, as IEEE bits under an atomic max (monotone for
// non-negative values, NaN the largest pattern).  Grid (ceil(d / 256), items,
// 2): z = 0 columns, z = 1 rows (a wave per row, so that the reads are coalesced).
template <typename C2>
__global__ __launch_bounds__(256) void shifted_norms_kernel(const C2* __restrict__ X, int d, int64_t b0,
                                                            const double2* __restrict__ mu,
                                                            unsigned long long* __restrict__ norms) {
  const int64_t b = b0 + blockIdx.y;
  const C2* A = X + b * d * d;
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

// norms[2 (b0 + b) + 1] = max row sum of |Omega - mu I| for item b0 + b
// (IEEE bits, atomic max).  A wave per row, eight loads in flight per lane;
// grid (ceil(d / 4), items).  For a skew-Hermitian matrix the max row sum is
// also the max column sum, so this one pass gives the 1-norm as well.
template <typename C2>
__global__ __launch_bounds__(256) void shifted_rownorm_kernel(const C2* __restrict__ X, int d, int64_t b0,
                                                              const double2* __restrict__ mu,
                                                              unsigned long long* __restrict__ norms) {
  const int64_t b = b0 + blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + wave;
  const double2 m = mu[b];
  double sum = 0.0;
  if (r < d) {
    const C2* ar = X + b * d * d + int64_t(r) * d;
    int c = lane;
    for (; c + 448 < d; c += 512) {
      C2 u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] = ar[c + 64 * q];
#pragma unroll
      for (int q = 0; q < 8; ++q) sum += shifted_abs(double(u[q].x), double(u[q].y), r == c + 64 * q, m);
    }
    for (; c < d; c += 64) {
      const C2 u = ar[c];
      sum += shifted_abs(double(u.x), double(u.y), r == c, m);
    }
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  __shared__ double red[4];
  if (lane == 0) red[wave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double best = red[0];
    nan_max(best, red[1]);
    nan_max(best, red[2]);
    nan_max(best, red[3]);
    atomicMax(norms + 2 * b + 1, (unsigned long long)__double_as_longlong(best));
  }
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

// ------------------------------------------------ half-read Taylor term
//
// Omega is skew-Hermitian (Omega_ji = -conj(Omega_ij), exactly so for the
// generators of Hermitian H0, H_k), so a product needs only its upper triangle:
// a 64 x 64 tile (I, J), I < J, gives its own rows' share y_I += Omega_IJ x_J
// and the mirrored tile's share y_J += -Omega_IJ^dag x_I; diagonal tiles are read
// whole.  Shares land in P[K][L][0..63] (K the output block, L the partner
// tile), so every output block has exactly nb shares, summed in a fixed order
// whatever order the tiles finish in (the result does not depend on
// scheduling).  HBM traffic per product: d (d + 64) / 2 elements of
// Omega instead of d^2.
constexpr int kActTile = 64;

// Tile t of the upper triangle, enumerated column by column: t = J (J + 1) / 2 + I.
__device__ __forceinline__ void action_tile_of(int t, int& I, int& J) {
  int j = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > t) --j;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  J = j;
  I = t - j * (j + 1) / 2;
}

// Finish 16 rows of output block K = blockIdx.x / 4: sum the nb shares in a
// fixed order (sixteen strided partial sums, four independent loads in flight
// per thread, combined in index order) and apply the term update of
// action_term_kernel.  Grid 4 nb, 256 threads.
__global__ __launch_bounds__(256) void action_finish_kernel(int d, int nb, const double2* __restrict__ x,
                                                            double2* __restrict__ y, double2* __restrict__ F,
                                                            const double2* __restrict__ P, double coef, double2 mu,
                                                            int last, double2 eta) {
  __shared__ double2 part[16][17];
  const int K = blockIdx.x >> 2, sub = blockIdx.x & 3;
  const int t = threadIdx.x & 15, p = threadIdx.x >> 4;
  const double2* src = P + int64_t(K) * nb * kActTile + 16 * sub + t;
  const int row = K * kActTile + 16 * sub + t;
  // the state rows go out with the shares (one round trip, not two)
  const bool upd = p == 0 && row < d;
  double2 xr = make_double2(0.0, 0.0), f = make_double2(0.0, 0.0);
  if (upd) {
    xr = x[row];
    f = F[row];
  }
  double sr = 0.0, si = 0.0;
  int L = p;
  for (; L + 48 < nb; L += 64) {
    double2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = src[int64_t(L + 16 * q) * kActTile];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sr += v[q].x;
      si += v[q].y;
    }
  }
  for (; L < nb; L += 16) {
    const double2 v = src[int64_t(L) * kActTile];
    sr += v.x;
    si += v.y;
  }
  part[p][t] = make_double2(sr, si);
  __syncthreads();
  if (upd) {
    sr = 0.0;
    si = 0.0;
#pragma unroll
    for (int g = 0; g < 16; ++g) {
      sr += part[g][t].x;
      si += part[g][t].y;
    }
    sr -= mu.x * xr.x - mu.y * xr.y;
    si -= mu.x * xr.y + mu.y * xr.x;
    const double2 tv = make_double2(coef * sr, coef * si);
    f.x += tv.x;
    f.y += tv.y;
    if (last) {
      f = make_double2(eta.x * f.x - eta.y * f.y, eta.x * f.y + eta.y * f.x);
      y[row] = f;
    } else {
      y[row] = tv;
    }
    F[row] = f;
  }
}

// One tile per workgroup (grid nb (nb + 1) / 2), writing its shares; the output
// blocks are finished by action_finish_kernel in a launch of its own (a
// last-workgroup-finishes variant needs device-wide fences that cost more than
// the launch).  A thread holds two adjacent columns of eight rows (rows rg,
// rg + 8, ...), so that a half-wave reads a whole 64-element row segment.
template <typename C2>
__global__ __launch_bounds__(256) void action_tile_kernel(const C2* __restrict__ A, int d, int nb,
                                                          const double2* __restrict__ x, double2* __restrict__ P) {
  int I, J;
  action_tile_of(int(blockIdx.x), I, J);
  const int tid = threadIdx.x, cp = tid & 31, rg = tid >> 5;
  const int r0 = I * kActTile, c0 = J * kActTile;
  const bool offdiag = I != J;
  __shared__ double2 xs[2][kActTile];
  __shared__ double2 colp[4][kActTile];
  // the tile's loads go out first (kept in the storage type until the
  // arithmetic); x comes from L2 meanwhile
  using R = decltype(C2::x);
  R rar[8][2], rai[8][2];
  const bool full = r0 + kActTile <= d && c0 + kActTile <= d;
  if (sizeof(C2) == 8 && full && (d & 1) == 0) {
    // complex64, even d: the two elements are one aligned 16-byte load
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float4 u = *reinterpret_cast<const float4*>(A + int64_t(r0 + rg + 8 * k) * d + c0 + 2 * cp);
      rar[k][0] = u.x;
      rai[k][0] = u.y;
      rar[k][1] = u.z;
      rai[k][1] = u.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int row = r0 + rg + 8 * k;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int col = c0 + 2 * cp + e;
        C2 v;
        v.x = 0;
        v.y = 0;
        if (full || (row < d && col < d)) v = A[int64_t(row) * d + col];
        rar[k][e] = v.x;
        rai[k][e] = v.y;
      }
    }
  }
  if (tid < 64) xs[0][tid] = r0 + tid < d ? x[r0 + tid] : make_double2(0.0, 0.0);
  else if (tid < 128) xs[1][tid - 64] = c0 + tid - 64 < d ? x[c0 + tid - 64] : make_double2(0.0, 0.0);
  __syncthreads();
  double ar[8][2], ai[8][2];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      ar[k][e] = double(rar[k][e]);
      ai[k][e] = double(rai[k][e]);
    }
  const double2 xc[2] = {xs[1][2 * cp], xs[1][2 * cp + 1]};
  double vr[8], vi[8];
  double csr[2] = {0.0, 0.0}, csi[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    vr[k] = 0.0;
    vi[k] = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      vr[k] += ar[k][e] * xc[e].x - ai[k][e] * xc[e].y;
      vi[k] += ar[k][e] * xc[e].y + ai[k][e] * xc[e].x;
    }
    if (offdiag) {
      // -conj(a) x_I[row]
      const double2 xr = xs[0][rg + 8 * k];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        csr[e] += -ar[k][e] * xr.x - ai[k][e] * xr.y;
        csi[e] += ai[k][e] * xr.x - ar[k][e] * xr.y;
      }
    }
  }
  // Row shares: the 32 lanes of a half-wave hold the same eight rows.  Recursive
  // halving over lane bits 4, 3, 2 (each lane keeps half of its rows and adds
  // its partner's half), then bits 1 and 0: lane 4 i of the half-wave ends with
  // the sum for row rg + 8 (4 b4 + 2 b3 + b2).
  const int lane = tid & 63;
  {
    const bool b = lane & 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double sr = b ? vr[i] : vr[4 + i], si = b ? vi[i] : vi[4 + i];
      const double kr = b ? vr[4 + i] : vr[i], ki = b ? vi[4 + i] : vi[i];
      vr[i] = kr + __shfl_xor(sr, 16);
      vi[i] = ki + __shfl_xor(si, 16);
    }
  }
  {
    const bool b = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double sr = b ? vr[i] : vr[2 + i], si = b ? vi[i] : vi[2 + i];
      const double kr = b ? vr[2 + i] : vr[i], ki = b ? vi[2 + i] : vi[i];
      vr[i] = kr + __shfl_xor(sr, 8);
      vi[i] = ki + __shfl_xor(si, 8);
    }
  }
  {
    const bool b = lane & 4;
    const double sr = b ? vr[0] : vr[1], si = b ? vi[0] : vi[1];
    const double kr = b ? vr[1] : vr[0], ki = b ? vi[1] : vi[0];
    vr[0] = kr + __shfl_xor(sr, 4);
    vi[0] = ki + __shfl_xor(si, 4);
  }
  vr[0] += __shfl_xor(vr[0], 2);
  vi[0] += __shfl_xor(vi[0], 2);
  vr[0] += __shfl_xor(vr[0], 1);
  vi[0] += __shfl_xor(vi[0], 1);
  if ((lane & 3) == 0) {
    const int k = ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
    P[(int64_t(I) * nb + J) * kActTile + rg + 8 * k] = make_double2(vr[0], vi[0]);
  }
  if (offdiag) {
    // column shares: the two half-waves of a wave, then the four waves in LDS
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      csr[e] += __shfl_xor(csr[e], 32);
      csi[e] += __shfl_xor(csi[e], 32);
    }
    if (lane < 32) {
      colp[tid >> 6][2 * cp] = make_double2(csr[0], csi[0]);
      colp[tid >> 6][2 * cp + 1] = make_double2(csr[1], csi[1]);
    }
    __syncthreads();
    if (tid < 64) {
      const double sr = ((colp[0][tid].x + colp[1][tid].x) + colp[2][tid].x) + colp[3][tid].x;
      const double si = ((colp[0][tid].y + colp[1][tid].y) + colp[2][tid].y) + colp[3][tid].y;
      P[(int64_t(J) * nb + I) * kActTile + tid] = make_double2(sr, si);
    }
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
