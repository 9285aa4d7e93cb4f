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

// Largest of a wave's 64 values, in every lane.  The partner of each step is
// taken through DPP moves within rows of 16 lanes (swap neighbours, swap pairs,
// mirror the half row, mirror the row), then the four row maxima are read out.
__device__ __forceinline__ double dpp_max_step(double v, int ctrl_id) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int plo, phi;
  switch (ctrl_id) {
    case 0: plo = __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false);
            phi = __builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: plo = __builtin_amdgcn_update_dpp(lo, lo, 0x4E, 0xF, 0xF, false);
            phi = __builtin_amdgcn_update_dpp(hi, hi, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: plo = __builtin_amdgcn_update_dpp(lo, lo, 0x141, 0xF, 0xF, false);
            phi = __builtin_amdgcn_update_dpp(hi, hi, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    default: plo = __builtin_amdgcn_update_dpp(lo, lo, 0x140, 0xF, 0xF, false);
             phi = __builtin_amdgcn_update_dpp(hi, hi, 0x140, 0xF, 0xF, false); break; // row_mirror
  }
  return fmax(v, __hiloint2double(phi, plo));
}

__device__ __forceinline__ double wave_max(double v) {
  v = dpp_max_step(v, 0);
  v = dpp_max_step(v, 1);
  v = dpp_max_step(v, 2);
  v = dpp_max_step(v, 3);
  // every lane of a row of 16 now holds that row's maximum
  double m = v;
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 16 * r);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 16 * r);
    m = fmax(m, __hiloint2double(hi, lo));
  }
  const int lo = __builtin_amdgcn_readlane(__double2loint(m), 0);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(m), 0);
  return __hiloint2double(hi, lo);
}

// Panel factorization of columns [k0, k1) (k1 - k0 <= NB) over rows [k0, d),
// d - k0 <= 1024, held in registers: thread t owns row k0 + t.  Pivot: the
// largest |re| + |im| in the column (compared on its leading 54 bits), ties to
// the lowest row.  Swaps the panel columns only; piv[k0 + j] = row exchanged with
// row k0 + j.
//
// The time of a column is a chain of LDS round trips that every wave walks at
// once (the barrier lines them up, so no wave hides another's latency); the
// kernel keeps that chain short:
//  - each wave reduces its candidates (DPP), then its winning lane publishes the
//    row and folds a 64-bit key (magnitude bits above, 1023 - row below) into
//    one LDS word with an atomic max, so after the single barrier per column a
//    thread reads one word to know the pivot;
//  - the pivot row is read in batches of eight (a sched barrier keeps the reads
//    issued together) rather than value by value;
//  - the pivot indices collect in LDS and go to memory after the last column.
// The keys rotate through three words: a column's word is cleared before the
// previous column's barrier, after the last read of the column that used it.
// The published rows alternate between two sets by column parity, so a column's
// writes never meet the previous column's reads.  The column loop is unrolled
// through Unroll so that every index into r[] is a compile-time constant and r
// stays in registers.
__device__ __forceinline__ unsigned long long pivot_key(double mag, int row) {
  return (static_cast<unsigned long long>(__double_as_longlong(mag)) & ~0x3FFull) |
         static_cast<unsigned long long>(1023 - row);
}

template <int NB>
__global__ __launch_bounds__(1024) void lu_panel_reg_kernel(double2* aug, int64_t ld, int64_t stride, int d, int k0,
                                                            int k1, int* piv_all) {
  constexpr int T = 1024, W = T / 64;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double2* A = aug + b * stride;
  int* piv = piv_all + int64_t(b) * d;
  const int nrows = d - k0, nc = k1 - k0;
  const bool own = tid < nrows;
  __shared__ unsigned long long key[3];
  __shared__ double2 wrow[2][W][NB];
  __shared__ double2 jrow[2][NB];
  __shared__ int spiv[NB];
  double2 r[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    r[c] = (own && c < nc) ? A[int64_t(k0 + tid) * ld + k0 + c] : make_double2(0.0, 0.0);
  if (tid < 3) key[tid] = 0ull;
  __syncthreads();

  Unroll<0, NB>::run([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    constexpr int par = j & 1;
    if (j >= nc) return;  // uniform across the workgroup
    const bool cand = own && tid >= j;
    const double v = cand ? pivot_mag(r[j]) : -1.0;
    const double m = wave_max(v);
    const unsigned long long hit = __ballot(cand && v == m);
    if (tid == 0) key[(j + 1) % 3] = 0ull;
    if (hit) {
      const int wl = __ffsll(static_cast<long long>(hit)) - 1;   // the lowest lane holding the maximum
      if (lane == wl) {
        atomicMax(&key[j % 3], pivot_key(m, tid));
#pragma unroll
        for (int c = 0; c < NB; ++c) wrow[par][wave][c] = r[c];
      }
    }
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < NB; ++c) jrow[par][c] = r[c];
    }
    __syncthreads();
    const unsigned long long kw = key[j % 3];
    const int p0 = 1023 - int(kw & 0x3FFull);
    const int p = (kw != 0ull && p0 >= j && p0 < nrows) ? p0 : j;
    if (tid == 0) {
      spiv[j] = k0 + p;
      const double best = __longlong_as_double(static_cast<long long>(kw & ~0x3FFull));
      if (!(best > 0.0)) flag_status(STATUS_ZERO_PIVOT);   // the largest |re| + |im| (NaN counts as inf)
    }
    const double2* prow = (p == p0) ? wrow[par][p >> 6] : jrow[par];
    if (p != j) {
      if (tid == j) {
#pragma unroll
        for (int c = 0; c < NB; ++c) r[c] = prow[c];
      } else if (tid == p) {
#pragma unroll
        for (int c = 0; c < NB; ++c) r[c] = jrow[par][c];
      }
    }
    if (own && tid > j) {
      // 1 / prow[j] as conj / |.|^2 (one division)
      const double2 pj = prow[j];
      const double rden = 1.0 / (pj.x * pj.x + pj.y * pj.y);
      const double2 l = cmul(r[j], make_double2(pj.x * rden, -pj.y * rden));
      r[j] = l;
      // the rest of the pivot row in chunks of eight values whose reads are in
      // flight together (the row arrays leave room for no more)
      Unroll<0, (NB - 1 - j + 7) / 8>::run([&](auto qc) {
        constexpr int c0 = j + 1 + 8 * decltype(qc)::value;
        constexpr int n = (NB - c0 < 8) ? NB - c0 : 8;
        double2 pr[n];
#pragma unroll
        for (int c = 0; c < n; ++c) pr[c] = prow[c0 + c];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < n; ++c) {
          const double2 t = cmul(l, pr[c]);
          r[c0 + c].x -= t.x;
          r[c0 + c].y -= t.y;
        }
      });
    }
  });

  __syncthreads();
  if (tid < nc) piv[k0 + tid] = spiv[tid];
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

// Loads and stores of the element `off` bytes past p, p uniform across the wave.
// p passes through readfirstlane, which keeps it in scalar registers as it is:
// the compiler cannot fold the per-lane offset into it, and each access takes the
// scalar-base plus 32-bit vector-offset form instead of a 64-bit vector address
// per row.
typedef double gd2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) gd2 gd2_global;
__device__ __forceinline__ gd2_global* uniform_at(double2* p, uint32_t off) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
  auto* base = reinterpret_cast<__attribute__((address_space(1))) char*>((uint64_t(hi) << 32) | lo);
  return reinterpret_cast<gd2_global*>(base + off);
}
__device__ __forceinline__ double2 load_at(double2* p, uint32_t off) {
  const gd2 v = *uniform_at(p, off);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void store_at(double2* p, uint32_t off, double2 v) {
  gd2 w;
  w.x = v.x;
  w.y = v.y;
  *uniform_at(p, off) = w;
}

// X <- L^{-1} X for rows [r0, r0 + 32), L = unit lower part of the diagonal block
// A[r0:r0+32, r0:r0+32], columns [c0, c1); one thread per column, no per-row
// guard (the recursion cuts the rows into leaves of 32 from the top, so only the
// last leaf of a size that is not a multiple of 32 takes the ragged form below).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void trsm_lower_unit_kernel(
    double2* aug, int64_t ld, int64_t stride, int r0, int c0, int c1) {
  const int b = blockIdx.y;
  double2* A = aug + b * stride;
  __shared__ double2 L[kTrsmNb][kTrsmNb];
  for (int e = threadIdx.x; e < kTrsmNb * kTrsmNb; e += 256) {
    const int i = e / kTrsmNb, j = e % kTrsmNb;
    L[i][j] = (j < i) ? A[int64_t(r0 + i) * ld + r0 + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int c = c0 + blockIdx.x * 256 + threadIdx.x;
  if (c >= c1) return;
  // row bases are uniform (scalar registers) and the column a 32-bit byte offset,
  // so the 32 loads and stores need no per-row vector address
  const uint32_t off = uint32_t(c) * uint32_t(sizeof(double2));
  double2 x[kTrsmNb];
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j)
    x[j] = load_at(A + int64_t(r0 + j) * ld, off);
#pragma unroll
  for (int i = 1; i < kTrsmNb; ++i) {
    double2 acc = x[i];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      const double2 l = L[i][j];
      acc.x -= l.x * x[j].x - l.y * x[j].y;
      acc.y -= l.x * x[j].y + l.y * x[j].x;
    }
    x[i] = acc;
    // one row at a time: without the barrier the compiler hoists every LDS read
    // of L ahead and runs out of registers (x alone takes 128)
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j)
    store_at(A + int64_t(r0 + j) * ld, off, x[j]);
}

// Placement of the solution by the last leaves of the backward solve: besides
// the FP64 rows the recursion above still reads, each leaf writes its final
// rows of R (the right half, columns d .. 2d) in the chunk's element type O to
// item b's buffer u1 when its squaring count s is odd and positive, else u0,
// where the squarings start (O = void: no placement).
template <typename O> struct LuPlace {
  const int* s;
  O* u0;
  O* u1;
  int d;
};
template <typename O> __device__ __forceinline__ O narrow_c(double2 v);
template <> __device__ __forceinline__ float2 narrow_c<float2>(double2 v) { return make_float2(float(v.x), float(v.y)); }
template <> __device__ __forceinline__ double2 narrow_c<double2>(double2 v) { return v; }
template <typename O>
__device__ __forceinline__ O* place_base(const LuPlace<O>& pl, int b) {
  const int s = pl.s[b];
  return ((s > 0 && (s & 1)) ? pl.u1 : pl.u0) + int64_t(b) * pl.d * pl.d;
}

// X <- U^{-1} X for rows [r0, r0 + 32), U = upper part of the diagonal block
// (non-unit diagonal, its reciprocals kept in LDS), columns [c0, c1); one thread
// per column, no per-row guard.
template <typename O>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void trsm_upper_kernel(
    double2* aug, int64_t ld, int64_t stride, int r0, int c0, int c1, LuPlace<O> pl) {
  const int b = blockIdx.y;
  double2* A = aug + b * stride;
  __shared__ double2 Ub[kTrsmNb][kTrsmNb];
  for (int e = threadIdx.x; e < kTrsmNb * kTrsmNb; e += 256) {
    const int i = e / kTrsmNb, j = e % kTrsmNb;
    double2 v = make_double2(0.0, 0.0);
    if (j >= i) v = A[int64_t(r0 + i) * ld + r0 + j];
    Ub[i][j] = (j == i) ? crecip(v) : v;
  }
  __syncthreads();
  const int c = c0 + blockIdx.x * 256 + threadIdx.x;
  if (c >= c1) return;
  // row bases are uniform (scalar registers) and the column a 32-bit byte offset,
  // so the 32 loads and stores need no per-row vector address
  const uint32_t off = uint32_t(c) * uint32_t(sizeof(double2));
  double2 x[kTrsmNb];
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j)
    x[j] = load_at(A + int64_t(r0 + j) * ld, off);
#pragma unroll
  for (int i = kTrsmNb - 1; i >= 0; --i) {
    double2 acc = x[i];
#pragma unroll
    for (int j = i + 1; j < kTrsmNb; ++j) {
      const double2 u = Ub[i][j];
      acc.x -= u.x * x[j].x - u.y * x[j].y;
      acc.y -= u.x * x[j].y + u.y * x[j].x;
    }
    x[i] = cmul(acc, Ub[i][i]);
    __builtin_amdgcn_sched_barrier(0);   // one row at a time, as in the lower leaf
  }
#pragma unroll
  for (int j = 0; j < kTrsmNb; ++j)
    store_at(A + int64_t(r0 + j) * ld, off, x[j]);
  if constexpr (!std::is_void_v<O>) {
    O* dst = place_base(pl, b) + (c - pl.d);
#pragma unroll
    for (int j = 0; j < kTrsmNb; ++j) dst[int64_t(r0 + j) * pl.d] = narrow_c<O>(x[j]);
  }
}

// The same two leaves for fewer than 32 rows (the last leaf of a size that is not
// a multiple of 32), with a guard per row: X <- L^{-1} X, L unit lower.
__global__ __launch_bounds__(256) void trsm_lower_unit_ragged_kernel(double2* aug, int64_t ld, int64_t stride, int r0,
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

// X <- U^{-1} X, U upper with a non-unit diagonal, fewer than 32 rows.
template <typename O>
__global__ __launch_bounds__(256) void trsm_upper_ragged_kernel(double2* aug, int64_t ld, int64_t stride, int r0, int r1,
                                                         int c0, int c1, LuPlace<O> pl) {
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
  if constexpr (!std::is_void_v<O>) {
    O* dst = place_base(pl, b) + (c - pl.d);
#pragma unroll
    for (int j = 0; j < kTrsmNb; ++j)
      if (j < nb) dst[int64_t(r0 + j) * pl.d] = narrow_c<O>(x[j]);
  }
}

}  // namespace qcheff
