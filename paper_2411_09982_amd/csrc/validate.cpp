// Host-side argument checks and workspace sizes (see validate.hpp).
#include "validate.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/qcheff.h"

namespace qcheff {

size_t elem_bytes(int dtype) {
  return dtype == QCHEFF_C128 ? 16 : dtype == QCHEFF_C64 ? 8 : 0;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

Check check_coeffs(const void* u, int64_t K, int64_t N, double dt_sample, int64_t M, int order,
                   const void* c1, const void* c2) {
  if (order < 1 || order > 3) return Check::fail(QCHEFF_EINVAL, "order must be 1, 2 or 3");
  if (K < 1) return Check::fail(QCHEFF_EINVAL, "K must be >= 1");
  if (N < 1 || M < 1) return Check::fail(QCHEFF_EINVAL, "N and M must be >= 1");
  if (N % M != 0) return Check::fail(QCHEFF_EINVAL, "N must be a multiple of M");
  if (!finite_pos(dt_sample)) return Check::fail(QCHEFF_EINVAL, "dt_sample must be finite and > 0");
  if (!u || !c1) return Check::fail(QCHEFF_EINVAL, "u and c1 must not be NULL");
  if (order >= 2 && !c2) return Check::fail(QCHEFF_EINVAL, "c2 must not be NULL for order 2 or 3");
  if (order == 3 && K > kMaxControls3)
    return Check::fail(QCHEFF_EUNSUPPORTED, "the third-order term takes at most 3 controls");
  if (K > 4096 || N > (int64_t(1) << 40)) return Check::fail(QCHEFF_EINVAL, "K or N too large");
  return Check::ok();
}

size_t generators_ws_bytes(int64_t d, int64_t K, int order) {
  if (order == 2) return align256(size_t(n_c2(K)) * size_t(d) * size_t(d) * 16);
  // order 3: both bases and two scratch products
  if (order == 3) return align256(size_t(n_c2(K) + n_c3(K) + 2) * size_t(d) * size_t(d) * 16);
  return 0;
}

Check check_generators(const void* H0, const void* Hk, int64_t d, int64_t K, int op_dtype,
                       const void* c1, const void* c2, int64_t M, double dt_interval, int order,
                       int out_dtype, const void* omega, const void* ws, size_t ws_bytes,
                       unsigned flags) {
  if (order < 1 || order > 3) return Check::fail(QCHEFF_EINVAL, "order must be 1, 2 or 3");
  if (d < 1 || d > kMaxDim) return Check::fail(QCHEFF_EINVAL, "d must be in [1, 16384]");
  if (K < 1) return Check::fail(QCHEFF_EINVAL, "K must be >= 1");
  if (M < 0) return Check::fail(QCHEFF_EINVAL, "M must be >= 0");
  if (!std::isfinite(dt_interval)) return Check::fail(QCHEFF_EINVAL, "dt_interval must be finite");
  if (flags & ~QCHEFF_REUSE_BASIS) return Check::fail(QCHEFF_EINVAL, "unknown flag bits");
  if (elem_bytes(op_dtype) == 0 || elem_bytes(out_dtype) == 0)
    return Check::fail(QCHEFF_EINVAL, "unknown dtype");
  if (op_dtype != QCHEFF_C128) return Check::fail(QCHEFF_EUNSUPPORTED, "operators must be QCHEFF_C128");
  if (K > kMaxControls) return Check::fail(QCHEFF_EUNSUPPORTED, "at most 8 controls");
  if (order == 3 && K > kMaxControls3)
    return Check::fail(QCHEFF_EUNSUPPORTED, "the third-order term takes at most 3 controls");
  if (!H0 || !Hk) return Check::fail(QCHEFF_EINVAL, "H0 and Hk must not be NULL");
  if (M > 0 && (!c1 || !omega)) return Check::fail(QCHEFF_EINVAL, "c1 and omega must not be NULL");
  if (order >= 2 && M > 0 && !c2) return Check::fail(QCHEFF_EINVAL, "c2 must not be NULL for order 2 or 3");
  if (order >= 2) {
    if (!ws) return Check::fail(QCHEFF_EWORKSPACE, "orders 2 and 3 need a workspace for the commutator basis");
    if (ws_bytes < generators_ws_bytes(d, K, order))
      return Check::fail(QCHEFF_EWORKSPACE, "workspace too small for the commutator basis");
  }
  return Check::ok();
}

// expm workspace, per item: six d x d matrices in dtype (A, A^2, A^4, A^6, W, V),
// one d x 2d augmented system in C128, d pivots (int32).
// Header: per-item FP64 norm slot, int32 squaring count.
size_t expm_item_bytes(int64_t d, int dtype) {
  size_t dd = size_t(d) * size_t(d);
  return 6 * align256(dd * elem_bytes(dtype)) + align256(2 * dd * 16) + align256(size_t(d) * 4);
}

size_t expm_header_bytes(int64_t batch) {
  // norms, squaring counts, their maximum, trace shifts
  return align256(size_t(batch) * 8) + align256(size_t(batch) * 4) + 256 + align256(size_t(batch) * 16);
}

size_t expm_ws_bytes(int64_t batch, int64_t d, int dtype) {
  if (batch < 1 || d < 1 || elem_bytes(dtype) == 0) return 0;
  return expm_header_bytes(batch) + size_t(batch) * expm_item_bytes(d, dtype);
}

int64_t expm_chunk(size_t ws_bytes, int64_t batch, int64_t d, int dtype) {
  if (batch < 1) return 0;
  // largest c <= batch with expm_ws_bytes(c) <= ws_bytes
  size_t item = expm_item_bytes(d, dtype);
  int64_t c = int64_t(ws_bytes / (item ? item : 1));
  if (c > batch) c = batch;
  while (c > 0 && expm_ws_bytes(c, d, dtype) > ws_bytes) --c;
  return c;
}

Check check_expm(const void* omega, int64_t batch, int64_t d, int dtype, const void* U,
                 const void* ws, size_t ws_bytes, int out_dtype) {
  if (out_dtype == 0) out_dtype = dtype;
  if (batch < 0) return Check::fail(QCHEFF_EINVAL, "batch must be >= 0");
  if (d < 1 || d > kMaxDim) return Check::fail(QCHEFF_EINVAL, "d must be in [1, 16384]");
  if (elem_bytes(dtype) == 0) return Check::fail(QCHEFF_EINVAL, "unknown dtype");
  if (batch == 0) return Check::ok();
  if (!omega || !U) return Check::fail(QCHEFF_EINVAL, "omega and U must not be NULL");
  {
    // the same buffer (same element type), or two that do not overlap (U serves as scratch)
    const size_t dd = size_t(batch) * size_t(d) * size_t(d);
    const size_t ob = dd * elem_bytes(dtype), ub = dd * elem_bytes(out_dtype);
    const uintptr_t o = reinterpret_cast<uintptr_t>(omega), u = reinterpret_cast<uintptr_t>(U);
    const bool same = omega == U && out_dtype == dtype;
    if (!same && o < u + ub && u < o + ob)
      return Check::fail(QCHEFF_EINVAL, out_dtype == dtype ? "U must be omega itself or not overlap it"
                                                           : "a complex128 U must not overlap omega");
  }
  if (!ws) return Check::fail(QCHEFF_EWORKSPACE, "workspace must not be NULL");
  if (expm_chunk(ws_bytes, batch, d, dtype) < 1)
    return Check::fail(QCHEFF_EWORKSPACE, "workspace smaller than one item needs");
  return Check::ok();
}

Check check_expm_grouped(int G, const void* const* omega, const int64_t* batch, const int64_t* d, int dtype,
                         void* const* U, const void* ws, size_t ws_bytes, int out_dtype) {
  if (G < 1 || G > 8) return Check::fail(QCHEFF_EINVAL, "G must be in [1, 8]");
  if (!omega || !batch || !d || !U) return Check::fail(QCHEFF_EINVAL, "omega, batch, d and U must not be NULL");
  size_t need = 0;
  for (int g = 0; g < G; ++g) {
    // the per-group checks of qcheff_expm_batched, the workspace aside
    Check c = check_expm(omega[g], batch[g], d[g], dtype, U[g], ws ? ws : omega, ~size_t(0), out_dtype);
    if (c.status) return Check::fail(c.status, "group " + std::to_string(g) + ": " + c.message);
    if (batch[g] > 0 && d[g] > 32) need += expm_ws_bytes(1, d[g], dtype);
  }
  if (need > 0 && !ws) return Check::fail(QCHEFF_EWORKSPACE, "workspace must not be NULL");
  if (need > ws_bytes)
    return Check::fail(QCHEFF_EWORKSPACE, "workspace smaller than one item of every group with d > 32 needs");
  return Check::ok();
}

size_t propagate_ws_bytes(int64_t M, int64_t d, int dtype, int mode) {
  if (M < 0 || d < 1 || elem_bytes(dtype) == 0) return 0;
  if (mode == QCHEFF_STATE) return align256(size_t(2 * d) * 16);
  if (mode == QCHEFF_PRODUCT) {
    size_t mat = align256(size_t(d) * size_t(d) * elem_bytes(dtype));
    return size_t((M + 1) / 2 + (M + 3) / 4) * mat;
  }
  return 0;
}

Check check_propagate(const void* U, int64_t M, int64_t d, int dtype, int mode, const void* x,
                      const void* traj, const void* ws, size_t ws_bytes, bool ws_given) {
  if (mode != QCHEFF_STATE && mode != QCHEFF_PRODUCT) return Check::fail(QCHEFF_EINVAL, "unknown mode");
  if (M < 0) return Check::fail(QCHEFF_EINVAL, "M must be >= 0");
  if (d < 1 || d > kMaxDim) return Check::fail(QCHEFF_EINVAL, "d must be in [1, 16384]");
  if (elem_bytes(dtype) == 0) return Check::fail(QCHEFF_EINVAL, "unknown dtype");
  if (!x) return Check::fail(QCHEFF_EINVAL, "x must not be NULL");
  if (M > 0 && !U) return Check::fail(QCHEFF_EINVAL, "U must not be NULL");
  if (mode == QCHEFF_PRODUCT && traj) return Check::fail(QCHEFF_EINVAL, "traj is for QCHEFF_STATE only");
  size_t need = propagate_ws_bytes(M, d, dtype, mode);
  if (ws_given && M > 0 && need > 0 && (!ws || ws_bytes < need))
    return Check::fail(QCHEFF_EWORKSPACE, "workspace too small");
  return Check::ok();
}

Check check_propagate_batched(const void* U, int64_t B, int64_t M, int64_t d, int dtype, const void* x) {
  if (B < 0 || M < 0) return Check::fail(QCHEFF_EINVAL, "B and M must be >= 0");
  if (d < 1 || d > 2048) return Check::fail(QCHEFF_EINVAL, "d must be in [1, 2048] (the state sits in LDS)");
  if (elem_bytes(dtype) == 0) return Check::fail(QCHEFF_EINVAL, "unknown dtype");
  if (B > 0x7fffffff) return Check::fail(QCHEFF_EINVAL, "B too large");
  if (B > 0 && !x) return Check::fail(QCHEFF_EINVAL, "x must not be NULL");
  if (B > 0 && M > 0 && !U) return Check::fail(QCHEFF_EINVAL, "U must not be NULL");
  return Check::ok();
}

size_t action_ws_bytes(int64_t M, int64_t d) {
  if (M < 0 || d < 1) return 0;
  // two term vectors, the per-interval shift and the two norms per interval;
  // the 64-row shares of the tiled product ([nb][nb][64] complex128)
  const size_t nb = size_t((d + 63) / 64);
  return 2 * align256(size_t(d) * 16) + align256(size_t(M) * 16) + align256(size_t(M) * 16) +
         align256(nb * nb * 64 * 16);
}

Check check_action(const void* omega, int64_t M, int64_t d, int dtype, const void* x, double tol, const void* ws,
                   size_t ws_bytes) {
  if (M < 0) return Check::fail(QCHEFF_EINVAL, "M must be >= 0");
  if (M > 0x7fffffff) return Check::fail(QCHEFF_EINVAL, "M too large");
  if (d < 1 || d > kMaxDim) return Check::fail(QCHEFF_EINVAL, "d must be in [1, 16384]");
  if (elem_bytes(dtype) == 0) return Check::fail(QCHEFF_EINVAL, "unknown dtype");
  if (!x) return Check::fail(QCHEFF_EINVAL, "x must not be NULL");
  if (M > 0 && !omega) return Check::fail(QCHEFF_EINVAL, "omega must not be NULL");
  if (!(tol >= 0.0) || tol >= 1.0) return Check::fail(QCHEFF_EINVAL, "tol must be in [0, 1)");
  if (!ws || ws_bytes < action_ws_bytes(M, d)) return Check::fail(QCHEFF_EWORKSPACE, "workspace too small");
  return Check::ok();
}

size_t npad_ws_bytes(int64_t P, int64_t d) {
  if (P < 0 || d < 2) return 0;
  const size_t p = size_t(P > 0 ? P : 1);
  return align256(size_t(d) * 4) + align256(p * 32) + align256(p * 4) + align256(size_t((d + 3) / 4) * 16);
}

Check check_npad(const void* H, int64_t d, int dtype, int64_t P, const void* ptr, const void* ws, size_t ws_bytes) {
  if (d < 2 || d > (int64_t(1) << 17)) return Check::fail(QCHEFF_EINVAL, "d must be in [2, 131072]");
  if (dtype != QCHEFF_C128 && dtype != QCHEFF_C64) return Check::fail(QCHEFF_EINVAL, "unknown dtype");
  if (P < 0 || P > d / 2) return Check::fail(QCHEFF_EINVAL, "P must be in [0, d/2] (disjoint pairs)");
  if (!H) return Check::fail(QCHEFF_EINVAL, "H must not be NULL");
  if (P > 0 && !ptr) return Check::fail(QCHEFF_EINVAL, "pairs must not be NULL");
  if (!ws || ws_bytes < npad_ws_bytes(P, d)) return Check::fail(QCHEFF_EWORKSPACE, "workspace too small");
  return Check::ok();
}

size_t workspace_bytes(int fn, int64_t batch, int64_t d, int64_t K, int order, int dtype) {
  if (fn == QCHEFF_FN_NPAD) return elem_bytes(dtype) ? npad_ws_bytes(batch, d) : 0;
  if (d < 1 || d > kMaxDim) return 0;
  switch (fn) {
    case QCHEFF_FN_GENERATORS:
      if (K < 1 || order < 1 || order > 3 || (order == 3 && K > kMaxControls3)) return 0;
      return generators_ws_bytes(d, K, order);
    case QCHEFF_FN_EXPM:
      return expm_ws_bytes(batch, d, dtype == QCHEFF_C64_BF16X3 ? QCHEFF_C64 : dtype);
    case QCHEFF_FN_PROPAGATE:
      return propagate_ws_bytes(batch, d, dtype, order);
    case QCHEFF_FN_ACTION:
      return elem_bytes(dtype) ? action_ws_bytes(batch, d) : 0;
    default:
      return 0;
  }
}

}  // namespace qcheff
