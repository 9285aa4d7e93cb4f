// Launch of the batched complex GEMM: picks the kernel of the tile
// configuration (FP32 cfg 0 / 1 / 4 on FP32 MFMA, FP32 cfg 2 / 3 on split BF16
// MFMA, FP64 cfg 0 / 1 / 4) and records the timing instrumentation.
#pragma once

#include <type_traits>

#include "cgemm.hpp"
#include "cgemm_bf16x3.hpp"

namespace qcheff {

template <typename T, int CFG> void launch_tile(const GemmParams<T>& p, unsigned blocks, hipStream_t stream) {
  using G = GemmTile<T, CFG>;
  if constexpr (std::is_same_v<T, float> && CFG == 3)
    hipLaunchKernelGGL((cgemm_bf16x3_planes_kernel<G::BM, G::BN, G::WM, G::WN, G::NT>), dim3(blocks), dim3(G::NT), 0,
                       stream, p);
  else if constexpr (std::is_same_v<T, float> && CFG == 2)
    hipLaunchKernelGGL((cgemm_bf16x3_kernel<G::BM, G::BN, G::WM, G::WN, G::NT>), dim3(blocks), dim3(G::NT), 0, stream,
                       p);
  else if constexpr (sizeof(T) == 8 && (CFG == 0 || CFG == 1)) {
    if (p.mode == 1)
      hipLaunchKernelGGL((cgemm_kernel<T, G::BM, G::BN, G::BK, G::WM, G::WN, G::NT, G::WPE, 1>), dim3(blocks),
                         dim3(G::NT), 0, stream, p);
    else
      hipLaunchKernelGGL((cgemm_kernel<T, G::BM, G::BN, G::BK, G::WM, G::WN, G::NT, G::WPE>), dim3(blocks),
                         dim3(G::NT), 0, stream, p);
  } else
    hipLaunchKernelGGL((cgemm_kernel<T, G::BM, G::BN, G::BK, G::WM, G::WN, G::NT, G::WPE>), dim3(blocks), dim3(G::NT),
                       0, stream, p);
}

// Launch; `active` is the number of items that do work (squaring mode skips
// the others) and feeds the timing record's algorithmic flop and byte counts.
template <typename T>
hipError_t launch_cgemm(const GemmParams<T>& p, hipStream_t stream, int64_t active = -1) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return hipSuccess;
  if (p.lda * int64_t(p.M) >= (int64_t(1) << 31) || p.ldb * int64_t(p.K) >= (int64_t(1) << 31) ||
      p.ldc * int64_t(p.M) >= (int64_t(1) << 31))
    return hipErrorInvalidValue;
  if (p.herm && (p.M != p.N || p.tiles_m != p.tiles_n)) return hipErrorInvalidValue;
  // mode 1: FP64 kernels of cfg 0 / 1 only, square products of one matrix
  if (p.mode == 1 && (sizeof(T) != 8 || (p.cfg != 0 && p.cfg != 1) || p.M != p.N || p.N != p.K || !p.a32))
    return hipErrorInvalidValue;
  if (p.epi == EPI_C32 && !p.c32) return hipErrorInvalidValue;
  const int64_t tiles = p.herm ? int64_t(p.tiles_m) * (p.tiles_m + 1) / 2 : int64_t(p.tiles_m) * p.tiles_n;
  const int64_t blocks = tiles * p.batch;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (active < 0) active = p.batch;
  LaunchTimer tm;
  tm.begin(stream);
  if constexpr (std::is_same_v<T, float>) {
    if (p.cfg == 2) launch_tile<T, 2>(p, unsigned(blocks), stream);
    if (p.cfg == 3) launch_tile<T, 3>(p, unsigned(blocks), stream);
  }
  if (p.cfg == 1)
    launch_tile<T, 1>(p, unsigned(blocks), stream);
  else if (p.cfg == 4)
    launch_tile<T, 4>(p, unsigned(blocks), stream);
  else if (p.cfg == 0)
    launch_tile<T, 0>(p, unsigned(blocks), stream);
  const hipError_t e = hipGetLastError();
  if (tm.on) {
    const double mn = double(p.M) * p.N, es = double(sizeof(typename Cx<T>::t));
    // a (skew-)Hermitian result has M (M + 1) / 2 distinct entries
    const double outs = p.herm ? double(p.M) * (p.M + 1) / 2 : mn;
    const double flops = 8.0 * outs * double(p.K) * double(active);
    double elems = double(p.M) * p.K + double(p.K) * p.N + mn * (1 + p.nx + (p.beta != T(0) ? 1 : 0));
    double bytes = elems * es;
    if (p.epi == EPI_AUG) bytes += mn * 32.0;  // V is the generic M N term; two FP64 halves are written
    if (p.epi == EPI_OUT64) bytes += mn * 8.0; // the result is written in FP64 (X_0 counted with nx)
    if (p.mode == 1) bytes -= (double(p.M) * p.K + double(p.K) * p.N) * (es - 8.0);   // complex64 operands
    if (p.epi == EPI_C32) bytes -= mn * (es - 8.0);                                   // complex64 result
    const int kid = sizeof(T) == 8 ? KERNEL_GEMM_F64 : split_bf16_cfg(p.cfg) ? KERNEL_GEMM_BF16X3
                                                      : KERNEL_GEMM_F32;
    tm.end(stream, kid, flops, bytes * double(active));
  }
  return e;
}

}  // namespace qcheff
