// Numerical NPAD (arXiv 2411.09982, Sec. 3.2): two-level Givens rotations that
// eliminate couplings of a dense Hermitian H in place, H <- G H G^dag, G the
// product of the rotations of disjoint index pairs (gfx950).
//
// Rotation of the pair (i, j) (Eq. tls-ham): delta = (H_ii - H_jj)/2,
// g = |H_ij|, e = H_ij / g, r = sqrt(delta^2 + g^2); theta = arctan(g/delta) on the
// principal branch (the level order is kept; delta = 0 counts as positive), and
// with c = cos(theta/2) = sqrt((1 + |delta|/r)/2), s = sign(delta) g / (2 r c):
//   G_ii = c, G_ij = s e, G_ji = -s conj(e), G_jj = c.
// Parameters and updates are formed in FP64; complex64 matrices are rounded once
// at the store.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace qcheff {

// Pairs given to qcheff_npad_eliminate that overlap or leave [0, d): those pairs
// are left alone and qcheff_sync_status reports QCHEFF_EINVAL.
enum : unsigned { STATUS_BAD_PAIRS = 4u };

struct NpadRot {
  double c, s, er, ei;   // G_ii = G_jj = c, G_ij = s (er + i ei)
};

__device__ __forceinline__ bool pair_in_range(int64_t i, int64_t j, int64_t d) {
  return i >= 0 && j >= 0 && i < d && j < d && i != j;
}

// mark[k] counts the pairs that use index k (mark starts at zero).
__global__ void npad_mark_kernel(const int64_t* __restrict__ pairs, int64_t P, int64_t d, int* __restrict__ mark) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
  if (!pair_in_range(i, j, d)) return;
  atomicAdd(mark + i, 1);
  atomicAdd(mark + j, 1);
}

template <typename C2>
__global__ void npad_params_kernel(const C2* __restrict__ H, int64_t d, const int64_t* __restrict__ pairs, int64_t P,
                                   const int* __restrict__ mark, NpadRot* __restrict__ rot, int* __restrict__ active) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
  if (!pair_in_range(i, j, d) || mark[i] != 1 || mark[j] != 1) {
    active[p] = 0;
    flag_status(STATUS_BAD_PAIRS);
    return;
  }
  const double a = double(H[i * d + i].x), cc = double(H[j * d + j].x);
  const C2 b = H[i * d + j];
  const double br = double(b.x), bi = double(b.y);
  const double g = sqrt(br * br + bi * bi);
  NpadRot r{1.0, 0.0, 1.0, 0.0};
  if (g > 0.0) {
    const double delta = 0.5 * (a - cc);
    const double rr = sqrt(delta * delta + g * g);
    const double c = sqrt(0.5 * (1.0 + fabs(delta) / rr));
    const double sgn = delta >= 0.0 ? 1.0 : -1.0;
    r = NpadRot{c, sgn * g / (2.0 * rr * c), br / g, bi / g};
  } else if (g != g) {   // a NaN coupling: the rows and columns become NaN
    r = NpadRot{g, g, g, g};
    flag_status(STATUS_NONFINITE);
  }
  rot[p] = r;
  active[p] = 1;
}

template <typename C2> __device__ __forceinline__ double2 ld2(const C2& v) {
  return make_double2(double(v.x), double(v.y));
}

// Rows i and j of every active pair: (G H)_ik = c H_ik + s e H_jk,
// (G H)_jk = -s conj(e) H_ik + c H_jk.  Block (x: columns, y: pairs).
template <typename C2>
__global__ __launch_bounds__(256) void npad_rows_kernel(C2* __restrict__ H, int64_t d, const int64_t* __restrict__ pairs,
                                                        int64_t p0, const NpadRot* __restrict__ rot,
                                                        const int* __restrict__ active) {
  const int64_t p = p0 + blockIdx.y;
  if (!active[p]) return;
  const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
  const NpadRot r = rot[p];
  C2* Hi = H + i * d;
  C2* Hj = H + j * d;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < d; k += int64_t(gridDim.x) * blockDim.x) {
    const double2 x = ld2(Hi[k]), y = ld2(Hj[k]);
    const double2 se = make_double2(r.s * r.er, r.s * r.ei);
    const double2 ni = make_double2(r.c * x.x + se.x * y.x - se.y * y.y, r.c * x.y + se.x * y.y + se.y * y.x);
    // -s conj(e) x = -(se.x - i se.y) x
    const double2 nj = make_double2(-(se.x * x.x + se.y * x.y) + r.c * y.x, -(se.x * x.y - se.y * x.x) + r.c * y.y);
    Hi[k] = to_c2<C2>(ni.x, ni.y);
    Hj[k] = to_c2<C2>(nj.x, nj.y);
  }
}

// Columns i and j of every active pair, after the rows: (H G^dag)_ki =
// c H_ki + s conj(e) H_kj, (H G^dag)_kj = -s e H_ki + c H_kj.  With many pairs the
// threads run over the pairs of one row (neighbouring pairs touch neighbouring
// columns); with few, over the rows of one pair.
template <typename C2, bool PAIRS_FAST>
__global__ __launch_bounds__(256) void npad_cols_kernel(C2* __restrict__ H, int64_t d, const int64_t* __restrict__ pairs,
                                                        int64_t P, int64_t p0, const NpadRot* __restrict__ rot,
                                                        const int* __restrict__ active) {
  int64_t p, k0, kstep;
  if constexpr (PAIRS_FAST) {
    p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    k0 = blockIdx.y;
    kstep = gridDim.y;
    if (p >= P) return;
  } else {
    p = p0 + blockIdx.y;
    k0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    kstep = int64_t(gridDim.x) * blockDim.x;
  }
  if (!active[p]) return;
  const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
  const NpadRot r = rot[p];
  const double2 se = make_double2(r.s * r.er, r.s * r.ei);
  for (int64_t k = k0; k < d; k += kstep) {
    C2* row = H + k * d;
    const double2 x = ld2(row[i]), y = ld2(row[j]);
    // s conj(e) y
    const double2 ni = make_double2(r.c * x.x + se.x * y.x + se.y * y.y, r.c * x.y + se.x * y.y - se.y * y.x);
    // -s e x
    const double2 nj = make_double2(-(se.x * x.x - se.y * x.y) + r.c * y.x, -(se.x * x.y + se.y * x.x) + r.c * y.y);
    row[i] = to_c2<C2>(ni.x, ni.y);
    row[j] = to_c2<C2>(nj.x, nj.y);
  }
}

// Largest |H_ij|, i < j: one wave per row, the first column among equal
// magnitudes (a NaN counts as the largest); per-block winners, then one block.
struct Best {
  double m;
  int64_t idx;
};

__device__ __forceinline__ Best better(Best a, Best b) {
  const bool an = a.m != a.m, bn = b.m != b.m;
  if (an != bn) return an ? a : b;
  if (a.m != b.m && !an) return a.m > b.m ? a : b;
  return a.idx <= b.idx ? a : b;
}

__device__ __forceinline__ Best wave_best(Best v) {
  for (int off = 32; off > 0; off >>= 1) {
    Best o{__shfl_down(v.m, off), __shfl_down(v.idx, off)};
    v = better(v, o);
  }
  return v;
}

template <typename C2>
__global__ __launch_bounds__(256) void npad_largest_partial_kernel(const C2* __restrict__ H, int64_t d,
                                                                   Best* __restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = int64_t(blockIdx.x) * 4 + wave;
  Best v{-1.0, INT64_MAX};
  if (i < d) {
    const C2* row = H + i * d;
    for (int64_t j = i + 1 + lane; j < d; j += 64) {
      const C2 x = row[j];
      const double m = sqrt(double(x.x) * double(x.x) + double(x.y) * double(x.y));
      v = better(v, Best{m, i * d + j});
    }
  }
  v = wave_best(v);
  __shared__ Best sh[4];
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = better(better(sh[0], sh[1]), better(sh[2], sh[3]));
}

__global__ __launch_bounds__(256) void npad_largest_final_kernel(const Best* __restrict__ part, int64_t n, int64_t d,
                                                                 int64_t* __restrict__ ij, double* __restrict__ mag) {
  Best v{-1.0, INT64_MAX};
  for (int64_t b = threadIdx.x; b < n; b += blockDim.x) v = better(v, part[b]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  v = wave_best(v);
  __shared__ Best sh[4];
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const Best w = better(better(sh[0], sh[1]), better(sh[2], sh[3]));
    ij[0] = w.idx / d;
    ij[1] = w.idx % d;
    if (mag) mag[0] = w.m;
  }
}

}  // namespace qcheff
