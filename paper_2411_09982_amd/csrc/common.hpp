// Shared device helpers for the gfx950 (CDNA4) kernels of libqcheff_magnus.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcheff {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Interleaved complex element and the 16x16 MFMA accumulator of a real type.
template <typename T> struct Cx;
template <> struct Cx<float> { using t = float2; using acc = f32x4; };
template <> struct Cx<double> { using t = double2; using acc = f64x4; };

// One 16x16x4 real MFMA: D = A(16x4) B(4x16) + C.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of accumulator element i held by lane l (its column is l % 16).  The FP32
// and FP64 16x16x4 instructions lay their results out differently.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int i);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int i) { return 4 * (lane >> 4) + i; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int i) { return (lane >> 4) + 4 * i; }

// The hardware hands consecutive workgroups to the 8 XCDs in turn.  Remap the
// linear block index so that each XCD receives a contiguous range of logical
// tiles: tiles of one matrix then share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;
  if (bid >= per * kXcd) return bid;
  return (bid % kXcd) * per + bid / kXcd;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename C2> __device__ __forceinline__ C2 czero();
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }

// Sticky status of the kernels on this device, read and cleared by
// qcheff_sync_status: bit 0 a non-finite norm, bit 1 a zero pivot.
__device__ unsigned status_word;
// Where qcheff_sync_status's one-thread kernel leaves the word it took.
__device__ unsigned status_taken;
enum : unsigned { STATUS_NONFINITE = 1u, STATUS_ZERO_PIVOT = 2u };
__device__ __forceinline__ void flag_status(unsigned bits) { atomicOr(&status_word, bits); }

// Takes the status word and clears it in one atomic step, so that a flag set by
// a kernel on another stream in between is kept for the next call, not lost.
__global__ void take_status_kernel() { status_taken = atomicExch(&status_word, 0u); }

}  // namespace qcheff
