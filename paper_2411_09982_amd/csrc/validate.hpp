// Host-side argument checks and workspace sizes of the C ABI (include/qcheff.h).
//
// Plain C++ with no HIP dependency, so that it builds with g++ and is unit-tested
// on a machine without a GPU.  Every check runs before anything is enqueued.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

namespace qcheff {

constexpr int64_t kMaxDim = 16384;      // largest d accepted
constexpr int64_t kMaxControls = 8;     // largest K accepted by the generator kernel
constexpr int kLuBlock = 32;            // panel width of the batched LU

struct Check {
  int status = 0;        // QCHEFF_* status
  std::string message;   // set when status != 0
  static Check ok() { return {}; }
  static Check fail(int st, std::string m) { return {st, std::move(m)}; }
};

inline int64_t n_pairs(int64_t K) { return K * (K - 1) / 2; }
inline int64_t n_c2(int64_t K) { return K + n_pairs(K); }
// Third-order basis: the index triples (a, b, c) of {0..K}^3 with a <= c, not
// a = b = c (x_0 the drift), whose nested commutators [H_a,[H_b,H_c]] + [H_c,[H_b,H_a]]
// weight the third-order term; (K+1) K (K+3) / 2 of them.
inline int64_t n_c3(int64_t K) { return (K + 1) * K * (K + 3) / 2; }
constexpr int64_t kMaxControls3 = 3;    // largest K of the third-order term
// columns of the coefficient table c2 for `order` (second-order ones first)
inline int64_t n_c2_cols(int64_t K, int order) { return order == 3 ? n_c2(K) + n_c3(K) : order == 2 ? n_c2(K) : 0; }
size_t elem_bytes(int dtype);   // 16 for C128, 8 for C64, 0 otherwise

Check check_coeffs(const void* u, int64_t K, int64_t N, double dt_sample, int64_t M, int order,
                   const void* c1, const void* c2);
Check check_generators(const void* H0, const void* Hk, int64_t d, int64_t K, int op_dtype,
                       const void* c1, const void* c2, int64_t M, double dt_interval, int order,
                       int out_dtype, const void* omega, const void* ws, size_t ws_bytes,
                       unsigned flags);
// out_dtype: the element type of U (dtype, or QCHEFF_C128 for an FP64 result
// of the FP32 path); 0 means dtype.
Check check_expm(const void* omega, int64_t batch, int64_t d, int dtype, const void* U,
                 const void* ws, size_t ws_bytes, int out_dtype = 0);
// qcheff_expm_grouped: G in [1, 8], every group valid for qcheff_expm_batched
// (apart from the workspace), and the workspace at least one item of every
// group with d > 32 (dtype without flags, out_dtype of the results).
Check check_expm_grouped(int G, const void* const* omega, const int64_t* batch, const int64_t* d, int dtype,
                         void* const* U, const void* ws, size_t ws_bytes, int out_dtype);
// ws_given = false: the caller passes no workspace (the allocation-free entry
// point brings its own scratch), so the workspace checks are skipped.
Check check_propagate(const void* U, int64_t M, int64_t d, int dtype, int mode, const void* x,
                      const void* traj, const void* ws, size_t ws_bytes, bool ws_given = true);

Check check_propagate_batched(const void* U, int64_t B, int64_t M, int64_t d, int dtype, const void* x);
Check check_action(const void* omega, int64_t M, int64_t d, int dtype, const void* x, double tol, const void* ws,
                   size_t ws_bytes);

// Workspace layouts.  Each region starts on a 256-byte boundary.
size_t align256(size_t n);
size_t generators_ws_bytes(int64_t d, int64_t K, int order);
// expm: per-item bytes and the fixed header
size_t expm_item_bytes(int64_t d, int dtype);
size_t expm_header_bytes(int64_t batch);
size_t expm_ws_bytes(int64_t batch, int64_t d, int dtype);
int64_t expm_chunk(size_t ws_bytes, int64_t batch, int64_t d, int dtype);  // items per chunk, 0 if none fit
size_t propagate_ws_bytes(int64_t M, int64_t d, int dtype, int mode);
size_t action_ws_bytes(int64_t M, int64_t d);
// qcheff_npad_*: H, d >= 2, dtype, P >= 0 pairs (device; checked by the kernels),
// workspace of npad_ws_bytes(P, d).
size_t npad_ws_bytes(int64_t P, int64_t d);
Check check_npad(const void* H, int64_t d, int dtype, int64_t P, const void* ptr, const void* ws, size_t ws_bytes);

size_t workspace_bytes(int fn, int64_t batch, int64_t d, int64_t K, int order, int dtype);

}  // namespace qcheff
