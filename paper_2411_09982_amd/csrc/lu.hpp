// Batched LU with partial pivoting in FP64 complex, for the Pade denominator
// solve (V - U) R = (V + U) on the augmented systems [q | p] (d x 2d, row-major).
//
// Recursive formulation (left half, row interchanges and triangular solve on the
// right half, Schur-complement update, right half): the updates are large
// complex GEMMs on MFMA (cgemm_kernel<double>), and only the leaves touch
// individual columns.  Leaves:
//   - panel factorization of a narrow column block over all rows below it,
//     with the block held in registers (one workgroup per item);
//   - row interchanges of a column range (one thread per column);
//   - unit-lower and upper triangular solves on <= 32 rows (one thread per column).
#pragma once

#include <type_traits>

#include "common.hpp"

namespace qcheff {

constexpr int kTrsmNb = 32;   // rows handled by one triangular-solve leaf

__device__ __forceinline__ double2 crecip(double2 a) {
  const double den = a.x * a.x + a.y * a.y;
  return make_double2(a.x / den, -a.y / den);
}

// Calls f(std::integral_constant<int, J>) for J = J0 .. J1 - 1.
template <int J0, int J1> struct Unroll {
  template <class F> __device__ __forceinline__ static void run(F&& f) {
    f(std::integral_constant<int, J0>{});
    Unroll<J0 + 1, J1>::run(f);
  }
};
template <int J1> struct Unroll<J1, J1> {
  template <class F> __device__ __forceinline__ static void run(F&&) {}
};

// Pivot magnitude |re| + |im|; a NaN entry counts as +inf so that the pivot
// search is a total order and always names a valid row.
__device__ __forceinline__ double pivot_mag(double2 v) {
  const double m = fabs(v.x) + fabs(v.y);
  return (m == m) ? m : __longlong_as_double(0x7ff0000000000000LL);
}

__device__ __forceinline__ void argmax_combine(double& v, int& i, double ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

// Panel factorization of columns [k0, k1) (k1 - k0 <= NB) over rows [k0, d),
// d - k0 <= 1024, held in registers: thread t owns row k0 + t.  Pivot: largest
// |re| + |im| in the column, ties to the lowest row.  Swaps the panel columns
// only; piv[k0 + j] = row exchanged with row k0 + j.  The column loop is
// unrolled through Unroll so that every index into r[] is a compile-time
// constant and r stays in registers.
template <int NB>
__global__ __launch_bounds__(1024) void lu_panel_reg_kernel(double2* aug, int64_t ld, int64_t stride, int d, int k0,
                                                            int k1, int* piv_all) {
  constexpr int T = 1024;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double2* A = aug + b * stride;
  int* piv = piv_all + int64_t(b) * d;
  const int nrows = d - k0, nc = k1 - k0;
  const bool own = tid < nrows;
  __shared__ double2 prow[NB];   // the pivot row of the current column
  __shared__ double2 orow[NB];   // the row it displaces
  __shared__ double wv[T / 64];
  __shared__ int wi[T / 64];
  double2 r[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    r[c] = (own && c < nc) ? A[int64_t(k0 + tid) * ld + k0 + c] : make_double2(0.0, 0.0);

  Unroll<0, NB>::run([&r, tid, lane, wave, nrows, nc, own, piv, k0](auto jc) {
    constexpr int j = decltype(jc)::value;
    if (j >= nc) return;  // uniform across the workgroup
    double v = -1.0;
    int idx = 0x7fffffff;
    if (own && tid >= j) {
      v = pivot_mag(r[j]);
      idx = tid;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off);
      const int oi = __shfl_xor(idx, off);
      argmax_combine(v, idx, ov, oi);
    }
    if (lane == 0) { wv[wave] = v; wi[wave] = idx; }
    __syncthreads();
    v = wv[0];
    idx = wi[0];
#pragma unroll
    for (int w = 1; w < T / 64; ++w) argmax_combine(v, idx, wv[w], wi[w]);
    const int p = (idx >= j && idx < nrows) ? idx : j;
    if (tid == 0) {
      piv[k0 + j] = k0 + p;
      if (!(v > 0.0)) flag_status(STATUS_ZERO_PIVOT);   // v is the largest |re| + |im| (NaN counts as inf)
    }
    // one exchange through LDS: the pivot row is published (it becomes row j
    // and drives the elimination), row j goes to the pivot's owner.  Two
    // barriers per column: every read of wv, prow and orow of this column
    // happens before the next column's first barrier, every write after it.
    if (tid == p) {
#pragma unroll
      for (int c = 0; c < NB; ++c) prow[c] = r[c];
    }
    if (p != j && tid == j) {
#pragma unroll
      for (int c = 0; c < NB; ++c) orow[c] = r[c];
    }
    __syncthreads();
    if (p != j) {
      if (tid == j) {
#pragma unroll
        for (int c = 0; c < NB; ++c) r[c] = prow[c];
      }
      if (tid == p) {
#pragma unroll
        for (int c = 0; c < NB; ++c) r[c] = orow[c];
      }
    }
    if (own && tid > j) {
      const double2 l = cmul(r[j], crecip(prow[j]));
      r[j] = l;
#pragma unroll
      for (int c = j + 1; c < NB; ++c) {
        const double2 t = cmul(l, prow[c]);
        r[c].x -= t.x;
        r[c].y -= t.y;
      }
    }
  });

  if (own) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nc) A[int64_t(k0 + tid) * ld + k0 + c] = r[c];
  }
}

// Panel factorization of columns [k0, k1) (k1 - k0 <= 32) over rows [k0, d)
// through global memory, one workgroup per item (any d).
__global__ __launch_bounds__(256) void lu_panel_kernel(double2* aug, int64_t ld, int64_t stride, int d, int k0,
                                                       int k1, int* piv_all) {
  const int b = blockIdx.x;
  double2* A = aug + b * stride;
  int* piv = piv_all + int64_t(b) * d;
  const int tid = threadIdx.x;
  __shared__ double smax[256];
  __shared__ int sidx[256];
  __shared__ double2 prow[kTrsmNb];
  for (int j = k0; j < k1; ++j) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = j + tid; i < d; i += 256) {
      const double m = pivot_mag(A[int64_t(i) * ld + j]);
      if (m > best) { best = m; bi = i; }
    }
    smax[tid] = best;
    sidx[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        double v = smax[tid];
        int i = sidx[tid];
        argmax_combine(v, i, smax[tid + w], sidx[tid + w]);
        smax[tid] = v;
        sidx[tid] = i;
      }
      __syncthreads();
    }
    const int pr = (sidx[0] >= j && sidx[0] < d) ? sidx[0] : j;
    if (tid == 0) {
      piv[j] = pr;
      if (!(smax[0] > 0.0)) flag_status(STATUS_ZERO_PIVOT);
    }
    if (pr != j) {
      for (int c = k0 + tid; c < k1; c += 256) {
        const double2 t = A[int64_t(j) * ld + c];
        A[int64_t(j) * ld + c] = A[int64_t(pr) * ld + c];
        A[int64_t(pr) * ld + c] = t;
      }
    }
    __syncthreads();
    if (tid < k1 - j) prow[tid] = A[int64_t(j) * ld + j + tid];
    __syncthreads();
    const double2 inv = crecip(prow[0]);
    for (int i = j + 1 + tid; i < d; i += 256) {
      double2* row = A + int64_t(i) * ld;
      const double2 l = cmul(row[j], inv);
      row[j] = l;
      for (int c = 1; c < k1 - j; ++c) {
        const double2 t = cmul(l, prow[c]);
        row[j + c].x -= t.x;
        row[j + c].y -= t.y;
      }
    }
    __syncthreads();
  }
}

// Row interchanges piv[k0..k1) applied in order to columns [c0, c1).
__global__ __launch_bounds__(256) void lu_pivots_kernel(double2* aug, int64_t ld, int64_t stride, int d, int k0,
                                                        int k1, int c0, int c1, const int* piv_all) {
  const int b = blockIdx.y;
  const int c = c0 + blockIdx.x * 256 + threadIdx.x;
  if (c >= c1) return;
  double2* A = aug + b * stride;
  const int* piv = piv_all + int64_t(b) * d;
  for (int j = k0; j < k1; ++j) {
    const int pr = piv[j];
    if (pr != j && pr >= 0 && pr < d) {
      const double2 t = A[int64_t(j) * ld + c];
      A[int64_t(j) * ld + c] = A[int64_t(pr) * ld + c];
      A[int64_t(pr) * ld + c] = t;
    }
  }
}

// X <- L^{-1} X for rows [r0, r1) (<= 32), L = unit lower part of A[r0:r1, r0:r1],
// columns [c0, c1); one thread per column.
__global__ __launch_bounds__(256) void trsm_lower_unit_kernel(double2* aug, int64_t ld, int64_t stride, int r0,
                                                              int r1, int c0, int c1) {
  const int b = blockIdx.y;
  double2* A = aug + b * stride;
  const int nb = r1 - r0;
  __shared__ double2 L[kTrsmNb][kTrsmNb + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    L[i][j] = A[int64_t(r0 + i) * ld + r0 + j];
  }
  __syncthreads();
  const int c = c0 + blockIdx.x * 256 + threadIdx.x;
  if (c >= c1) return;
  double2 x[kTrsmNb];
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j) x[j] = (j < nb) ? A[int64_t(r0 + j) * ld + c] : make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j) {
#pragma unroll
    for (int i = j + 1; i < kTrsmNb; ++i) {
      if (i < nb) {
        const double2 t = cmul(L[i][j], x[j]);
        x[i].x -= t.x;
        x[i].y -= t.y;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j)
    if (j < nb) A[int64_t(r0 + j) * ld + c] = x[j];
}

// X <- U^{-1} X for rows [r0, r1) (<= 32), U = upper part of A[r0:r1, r0:r1]
// (non-unit diagonal), columns [c0, c1); one thread per column.
__global__ __launch_bounds__(256) void trsm_upper_kernel(double2* aug, int64_t ld, int64_t stride, int r0, int r1,
                                                         int c0, int c1) {
  const int b = blockIdx.y;
  double2* A = aug + b * stride;
  const int nb = r1 - r0;
  __shared__ double2 Ub[kTrsmNb][kTrsmNb + 1];
  __shared__ double2 Dinv[kTrsmNb];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    Ub[i][j] = (j >= i) ? A[int64_t(r0 + i) * ld + r0 + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (threadIdx.x < nb) Dinv[threadIdx.x] = crecip(Ub[threadIdx.x][threadIdx.x]);
  __syncthreads();
  const int c = c0 + blockIdx.x * 256 + threadIdx.x;
  if (c >= c1) return;
  double2 x[kTrsmNb];
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j) x[j] = (j < nb) ? A[int64_t(r0 + j) * ld + c] : make_double2(0.0, 0.0);
#pragma unroll
  for (int i = kTrsmNb - 1; i >= 0; --i) {
    if (i < nb) {
      double2 v = x[i];
#pragma unroll
      for (int j = i + 1; j < kTrsmNb; ++j) {
        if (j < nb) {
          const double2 t = cmul(Ub[i][j], x[j]);
          v.x -= t.x;
          v.y -= t.y;
        }
      }
      x[i] = cmul(v, Dinv[i]);
    }
  }
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j)
    if (j < nb) A[int64_t(r0 + j) * ld + c] = x[j];
}

}  // namespace qcheff
