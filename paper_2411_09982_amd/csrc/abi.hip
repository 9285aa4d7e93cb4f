// C ABI of libqcheff_magnus (include/qcheff.h): argument checks, workspace
// carving and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <cstring>
#include <vector>

#include "../../include/qcheff.h"
#include "gemm_launch.hpp"
#include "kernels.hpp"
#include "lu.hpp"
#include "expm_small.hpp"
#include "action.hpp"
#include "npad.hpp"
#include "validate.hpp"

namespace qcheff {

// ------------------------------------------------------------- timing
namespace {
struct TimedLaunch {
  int kernel;
  double flops, bytes;
  hipEvent_t a, b;
};
std::atomic<int> g_timing{0};
// Conditions found on the host (per device), reported with the device's own.
constexpr int kMaxDevices = 64;
std::atomic<unsigned> g_host_status[kMaxDevices];
std::mutex g_status_mu;   // one take-and-copy of the device status word at a time

void flag_host_status(unsigned bits) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  g_host_status[dev].fetch_or(bits);
}
std::mutex g_timing_mu;               // guards g_timed and g_events
std::vector<TimedLaunch> g_timed;
// Events come from a pool and go back to it once read: creating two events per
// launch costs more host time than some of the launches they time.
std::vector<hipEvent_t> g_events;

hipError_t take_event(hipEvent_t* e) {
  {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (!g_events.empty()) {
      *e = g_events.back();
      g_events.pop_back();
      return hipSuccess;
    }
  }
  return hipEventCreate(e);
}

void give_events_locked(const TimedLaunch& t) {
  g_events.push_back(t.a);
  g_events.push_back(t.b);
}
}  // namespace

void LaunchTimer::begin(hipStream_t st) {
  on = g_timing.load(std::memory_order_relaxed) != 0;
  if (!on) return;
  if (take_event(&a) != hipSuccess) {
    on = false;
    return;
  }
  if (take_event(&b) != hipSuccess || hipEventRecord(a, st) != hipSuccess) {
    on = false;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_events.push_back(a);
    if (b) g_events.push_back(b);
  }
}

void LaunchTimer::end(hipStream_t st, int kernel, double flops, double bytes) {
  if (!on) return;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (hipEventRecord(b, st) != hipSuccess) {
    g_events.push_back(a);
    g_events.push_back(b);
    return;
  }
  g_timed.push_back({kernel, flops, bytes, a, b});
}

namespace {

thread_local std::string g_last_error = "no error";

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int fail(const Check& c) { return fail(c.status, c.message); }

#define QC_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(QCHEFF_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_));   \
  } while (0)

inline unsigned nblocks(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// Carves a workspace into 256-byte aligned regions.
struct Carver {
  char* p;
  size_t left;
  template <typename Tp> Tp* take(size_t bytes) {
    bytes = align256(bytes);
    if (bytes > left) return nullptr;
    Tp* r = reinterpret_cast<Tp*>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

// [m/m] Pade coefficients of exp: b_j = (2m-j)! m! / ((2m)! j! (m-j)!), b_0 = 1.
void pade_coefficients(int m, double* b) {
  b[0] = 1.0;
  for (int j = 0; j < m; ++j) b[j + 1] = b[j] * double(m - j) / (double(2 * m - j) * double(j + 1));
}

// Largest 1-norm for which the [13/13] approximant reaches double-precision
// backward error (Higham 2005, Table 2.3).  The FP32 path uses it too: its
// truncation error would allow about twice the norm, but the rounding error of
// evaluating the degree-13 polynomials in FP32 grows with sum_j b_j ||A||^j
// (about 15 at this norm, 270 at twice it), which costs more accuracy than the
// squaring it saves.
constexpr double kTheta13 = 5.371920351148152;

// -------------------------------------------------------------- tile tuner
//
// The square batched products of one exponential call all share a shape.  The
// first call for a (precision, d, Hermitian or not) triple times every tile
// configuration of kTunedCfgs on the chunk's own A*A product (for skew-Hermitian
// inputs its upper half and the whole product, summed; two launches of each,
// the second one timed with HIP events) and keeps the fastest for the rest of
// the process.  Every
// configuration accumulates each output element over k in the same order, so
// the choice changes speed only, never a bit of the result.
// QCHEFF_AUTOTUNE=0 replaces the timing with a size rule; QCHEFF_TUNE_FILE
// names a text file of "key d cfg" lines (key: the precision code, plus 100 for
// Hermitian-half products) read at first use and appended
// to after each new decision.
std::mutex g_tune_mu;
std::map<std::pair<int, int64_t>, int> g_tune;
constexpr int kTuneHermKey = 100;   // added to the precision code of Hermitian-half products
bool g_tune_loaded = false;

int rule_cfg(int64_t d) { return d <= 96 ? 1 : 0; }

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* f = std::getenv("QCHEFF_TUNE_FILE");
  if (!f) return;
  if (FILE* fp = std::fopen(f, "r")) {
    int prec, cfg;
    long long d;
    while (std::fscanf(fp, "%d %lld %d", &prec, &d, &cfg) == 3)
      if (cfg == 0 || cfg == 1 || cfg == 4) g_tune[{prec, int64_t(d)}] = cfg;
    std::fclose(fp);
  }
}

void tune_store_locked(int prec, int64_t d, int cfg) {
  g_tune[{prec, d}] = cfg;
  const char* f = std::getenv("QCHEFF_TUNE_FILE");
  if (!f) return;
  if (FILE* fp = std::fopen(f, "a")) {
    std::fprintf(fp, "%d %lld %d\n", prec, (long long)d, cfg);
    std::fclose(fp);
  }
}

template <typename T>
int square_cfg(int64_t d, int64_t nb, const typename Cx<T>::t* A, typename Cx<T>::t* scratch, bool herm,
               hipStream_t st, int* cfg_out) {
  // the key tells Hermitian-half products (skew-Hermitian inputs: all six Pade
  // products) from general ones: larger tiles lose more on the diagonal
  const int prec = (sizeof(T) == 8 ? QCHEFF_C128 : QCHEFF_C64) + (herm ? kTuneHermKey : 0);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find({prec, d});
    if (it != g_tune.end()) {
      *cfg_out = it->second;
      return QCHEFF_OK;
    }
  }
  const char* env = std::getenv("QCHEFF_AUTOTUNE");
  int best = rule_cfg(d);
  // Timing waits on the host, which a stream under graph capture must not do:
  // there the size rule stands in (and is not stored).
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  QC_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) {
    *cfg_out = best;
    return QCHEFF_OK;
  }
  if (!(env && env[0] == '0')) {
    float best_ms = 3.4e38f;
    hipEvent_t e0, e1;
    QC_HIP(hipEventCreate(&e0));
    QC_HIP(hipEventCreate(&e1));
    // the call's products as they come: with a Hermitian-half product first
    // (skew-Hermitian inputs: the six Pade products), then a general one (the
    // squarings); each timed after one untimed launch, the sum compared
    for (const int cfg : kTunedCfgs) {
      float total = 0.f;
      for (const int hm : {herm ? 1 : 0, 0}) {
        auto p = gemm_params<T>(int(d), int(d), int(d), int(nb), cfg);
        p.A = A; p.lda = d; p.sA = d * d;
        p.B = A; p.ldb = d; p.sB = d * d;
        p.C = scratch; p.ldc = d; p.sC = d * d;
        p.herm = hm;
        QC_HIP((launch_cgemm<T>(p, st, 0)));
        QC_HIP(hipEventRecord(e0, st));
        QC_HIP((launch_cgemm<T>(p, st, 0)));
        QC_HIP(hipEventRecord(e1, st));
        QC_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        QC_HIP(hipEventElapsedTime(&ms, e0, e1));
        total += ms;
        if (!herm) break;   // general products only
      }
      if (total < best_ms) { best_ms = total; best = cfg; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_store_locked(prec, d, best);
  *cfg_out = best;
  return QCHEFF_OK;
}

// The split-BF16 GEMM variant: the split done once per workgroup at the LDS
// store (cfg 3, the default: 181 algorithmic TFLOP/s on the d = 1000 job), or
// by each wave as it reads a fragment (cfg 2, QCHEFF_BF16X3_KERNEL=fragments:
// 158); both give the same bits.
int bf16x3_cfg() {
  const char* v = std::getenv("QCHEFF_BF16X3_KERNEL");
  return (v && std::strcmp(v, "fragments") == 0) ? 2 : 3;
}

// Taylor-term kernel: 0 reads Omega whole (a wave per row), 1 reads its upper
// triangle by tiles and finishes the output blocks in a second launch.  Below
// d = 2048 the tile grid (nb (nb + 1) / 2 workgroups) does not fill the chip.
// The tiles need generators declared skew-Hermitian (the lower triangle is not
// read); without the declaration every product reads the whole matrix.
int action_mode(int64_t d, bool skew) {
  if (!skew) return 0;
  const char* v = std::getenv("QCHEFF_ACTION_KERNEL");
  if (v && std::strcmp(v, "rows") == 0) return 0;
  if (v && std::strcmp(v, "tiles") == 0) return 1;
  return d >= 2048 ? 1 : 0;
}

// ------------------------------------------------- allocation-free entry
//
// qcheff_propagate_state_noalloc takes the scratch of the state chain (two
// ping-pong state vectors) from this file-scope device array instead of a
// caller workspace.  Each device holds its own copy; host code never passes
// the symbol itself to a kernel: it passes the address hipGetSymbolAddress
// returned for the current device (kept per device below).
constexpr int64_t kScratchVecs = 2 * kMaxDim;          // complex128 elements: 512 KiB
static __device__ __align__(256) double2 scratch[kScratchVecs];
std::mutex g_scratch_mu;
double2* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(double2** out) {
  int dev = 0;
  QC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(QCHEFF_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    QC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double2*>(p);
  }
  *out = g_scratch_ptr[dev];
  return QCHEFF_OK;
}

// ------------------------------------------------------------------- coeffs
int run_coeffs(const double* u, int64_t K, int64_t N, double dt, int64_t M, int order, double* c1,
               double* c2, hipStream_t st) {
  const int64_t s = N / M;
  const int ldc2 = int(n_c2_cols(K, order));
  // one wave per interval, four per workgroup
  hipLaunchKernelGGL(coeffs_kernel, dim3(nblocks(M, 4)), dim3(256), 0, st, u, int(K), N, M, s, dt, order, c1, c2,
                     ldc2);
  if (order == 3)
    hipLaunchKernelGGL(coeffs3_kernel, dim3(nblocks(M, 4)), dim3(256), 0, st, u, int(K), N, M, s, dt, ldc2,
                       int(n_c2(K)), c2);
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

// --------------------------------------------------------------- generators
template <int K, int ORDER, typename OutC2>
hipError_t launch_generators(const double2* H0, const double2* Hk, const double2* Cb, int64_t d,
                             const double* c1, const double* c2, int64_t M, double dt, OutC2* omega,
                             hipStream_t st) {
  constexpr int NC = K + ((ORDER >= 2) ? K + K * (K - 1) / 2 : 0) + ((ORDER == 3) ? (K + 1) * K * (K + 3) / 2 : 0);
  const int64_t dd = d * d;
  // A block reads its operator values once per chunk of nch intervals, so the
  // chunks are as long as 48 KB of coefficients allow, unless the grid would
  // then have fewer than 2048 blocks.
  const int64_t xb = int64_t(nblocks(dd, 256));
  const int64_t cap = std::min<int64_t>(256, 49152 / (NC * int64_t(sizeof(double))));
  const int64_t ych = std::max<int64_t>(1, (2048 + xb - 1) / xb);
  const int nch = int(std::max<int64_t>(1, std::min<int64_t>(cap, (M + ych - 1) / ych)));
  dim3 grid(unsigned(xb), unsigned((M + nch - 1) / nch));
  hipLaunchKernelGGL((generators_kernel<K, ORDER, OutC2>), grid, dim3(256), size_t(nch) * NC * sizeof(double), st,
                     H0, Hk, Cb, dd, c1, c2, M, nch, dt, omega);
  return hipGetLastError();
}

template <int ORDER, typename OutC2>
hipError_t dispatch_generators(int K, const double2* H0, const double2* Hk, const double2* Cb, int64_t d,
                               const double* c1, const double* c2, int64_t M, double dt, OutC2* omega,
                               hipStream_t st) {
  if constexpr (ORDER == 3) {   // the third-order term takes K <= 3
    switch (K) {
      case 1: return launch_generators<1, 3, OutC2>(H0, Hk, Cb, d, c1, c2, M, dt, omega, st);
      case 2: return launch_generators<2, 3, OutC2>(H0, Hk, Cb, d, c1, c2, M, dt, omega, st);
      case 3: return launch_generators<3, 3, OutC2>(H0, Hk, Cb, d, c1, c2, M, dt, omega, st);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (K) {
#define QC_CASE(k) \
  case k: return launch_generators<k, ORDER, OutC2>(H0, Hk, Cb, d, c1, c2, M, dt, omega, st);
      QC_CASE(1) QC_CASE(2) QC_CASE(3) QC_CASE(4) QC_CASE(5) QC_CASE(6) QC_CASE(7) QC_CASE(8)
#undef QC_CASE
      default: return hipErrorInvalidValue;
    }
  }
}

// [F, G] for Hermitian F, G into C: C = F G on MFMA (FP64), then C <- C - C^dag.
int commutator(const double2* F, const double2* G, double2* C, int64_t d, hipStream_t st) {
  auto p = gemm_params<double>(int(d), int(d), int(d), 1);
  p.A = reinterpret_cast<const double2*>(F); p.lda = d; p.sA = 0;
  p.B = reinterpret_cast<const double2*>(G); p.ldb = d; p.sB = 0;
  p.C = C; p.ldc = d; p.sC = 0;
  QC_HIP((launch_cgemm<double>(p, st)));
  hipLaunchKernelGGL(antihermitian_part_kernel, dim3(nblocks(d * d, 256)), dim3(256), 0, st, C, int(d));
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

// [H_b, H_c] from the second-order basis (0 is the drift): [H0, H_k] is basis
// entry k - 1, [H_k, H_l] (k < l) entry K + pair(k - 1, l - 1); [H_c, H_b] = -[H_b, H_c].
// Returns the entry and the sign, or sign 0 for b == c.
int comm_entry(int b, int c, int K, int* sign) {
  if (b == c) {
    *sign = 0;
    return 0;
  }
  *sign = b < c ? 1 : -1;
  const int lo = std::min(b, c), hi = std::max(b, c);
  if (lo == 0) return hi - 1;
  const int k = lo - 1, l = hi - 1;
  return K + k * K - k * (k + 1) / 2 + (l - k - 1);
}

int run_generators(const double2* H0, const double2* Hk, int64_t d, int64_t K, const double* c1,
                   const double* c2, int64_t M, double dt, int order, int out_dtype, void* omega,
                   void* ws, unsigned flags, hipStream_t st) {
  double2* Cb = static_cast<double2*>(ws);
  const int64_t dd = d * d;
  if (order >= 2 && !(flags & QCHEFF_REUSE_BASIS)) {
    int q = 0;
    for (int64_t k = 0; k < K; ++k, ++q) {
      int r = commutator(H0, Hk + k * dd, Cb + q * dd, d, st);
      if (r) return r;
    }
    for (int64_t k = 0; k < K; ++k)
      for (int64_t l = k + 1; l < K; ++l, ++q) {
        int r = commutator(Hk + k * dd, Hk + l * dd, Cb + q * dd, d, st);
        if (r) return r;
      }
    if (order == 3) {
      // [H_a, [H_b, H_c]] + [H_c, [H_b, H_a]] for the triples of the third-order term,
      // each [H, D] = H D + (H D)^dag formed from one FP64 product
      const int P2 = int(n_c2(K));
      double2* C3 = Cb + int64_t(P2) * dd;
      double2* X1 = C3 + n_c3(K) * dd;
      double2* X2 = X1 + dd;
      auto H = [&](int a) { return a == 0 ? H0 : Hk + int64_t(a - 1) * dd; };
      auto product = [&](int a, int b, int c, double2* X) -> int {   // X = H_a [H_b, H_c], or 0 if b == c
        int sign;
        const int ent = comm_entry(b, c, int(K), &sign);
        if (!sign) return 0;
        auto p = gemm_params<double>(int(d), int(d), int(d), 1);
        p.A = H(a); p.lda = d; p.sA = 0;
        p.B = Cb + int64_t(ent) * dd; p.ldb = d; p.sB = 0;
        p.C = X; p.ldc = d; p.sC = 0;
        p.alpha = double(sign);
        QC_HIP((launch_cgemm<double>(p, st)));
        return 1;
      };
      int t = 0;
      for (int a = 0; a <= K; ++a)
        for (int c = a; c <= K; ++c)
          for (int b = 0; b <= K; ++b) {
            if (a == b && b == c) continue;
            const int u1 = product(a, b, c, X1);
            if (u1 < 0) return u1;
            const int u2 = product(c, b, a, X2);
            if (u2 < 0) return u2;
            hipLaunchKernelGGL(hermitian_sum_kernel, dim3(nblocks(dd, 256)), dim3(256), 0, st, u1 ? X1 : nullptr,
                               u2 ? X2 : nullptr, C3 + int64_t(t) * dd, int(d));
            QC_HIP(hipGetLastError());
            ++t;
          }
    }
  }
  if (M == 0) return QCHEFF_OK;
  hipError_t e;
  if (out_dtype == QCHEFF_C128) {
    double2* om = static_cast<double2*>(omega);
    e = order == 3   ? dispatch_generators<3>(int(K), H0, Hk, Cb, d, c1, c2, M, dt, om, st)
        : order == 2 ? dispatch_generators<2>(int(K), H0, Hk, Cb, d, c1, c2, M, dt, om, st)
                     : dispatch_generators<1>(int(K), H0, Hk, Cb, d, c1, c2, M, dt, om, st);
  } else {
    float2* om = static_cast<float2*>(omega);
    e = order == 3   ? dispatch_generators<3>(int(K), H0, Hk, Cb, d, c1, c2, M, dt, om, st)
        : order == 2 ? dispatch_generators<2>(int(K), H0, Hk, Cb, d, c1, c2, M, dt, om, st)
                     : dispatch_generators<1>(int(K), H0, Hk, Cb, d, c1, c2, M, dt, om, st);
  }
  QC_HIP(e);
  return QCHEFF_OK;
}

// --------------------------------------------------------------------- expm

// Workspace regions of one expm chunk.
template <typename T> struct ExpmWs {
  using C2 = typename Cx<T>::t;
  unsigned long long* norms;
  int* s_ws;
  int* smax;
  double2* mu;   // trace shifts
  C2* X[6];
  double2* aug;
  int* piv;
};

template <typename T> bool carve_expm(void* ws, size_t bytes, int64_t chunk, int64_t d, ExpmWs<T>& w) {
  Carver cv{static_cast<char*>(ws), bytes};
  const size_t dd = size_t(d) * size_t(d);
  w.norms = cv.take<unsigned long long>(size_t(chunk) * 8);
  w.s_ws = cv.take<int>(size_t(chunk) * 4);
  w.smax = cv.take<int>(256);
  w.mu = cv.take<double2>(size_t(chunk) * 16);
  for (int i = 0; i < 6; ++i) w.X[i] = cv.take<typename Cx<T>::t>(size_t(chunk) * dd * sizeof(typename Cx<T>::t));
  w.aug = cv.take<double2>(size_t(chunk) * 2 * dd * 16);
  w.piv = cv.take<int>(size_t(chunk) * size_t(d) * 4);
  bool ok = w.norms && w.s_ws && w.smax && w.mu && w.aug && w.piv;
  for (int i = 0; i < 6; ++i) ok = ok && w.X[i];
  return ok;
}

// out = A B (+ sum_i xc[i] X_i + gamma I) over a batch of d x d items.
template <typename T>
int gemm_sq(int cfg, int herm, typename Cx<T>::t* out, const typename Cx<T>::t* A, const typename Cx<T>::t* B,
            int64_t d, int64_t nb, hipStream_t st, int nx = 0, const typename Cx<T>::t* const* X = nullptr,
            const T* xc = nullptr, T gamma = T(0)) {
  auto p = gemm_params<T>(int(d), int(d), int(d), int(nb), cfg);
  p.herm = herm;
  const int64_t dd = d * d;
  p.A = A; p.lda = d; p.sA = dd;
  p.B = B; p.ldb = d; p.sB = dd;
  p.C = out; p.ldc = d; p.sC = dd;
  p.nx = nx;
  for (int i = 0; i < nx; ++i) { p.X[i] = X[i]; p.xc[i] = xc[i]; }
  p.gamma = gamma;
  QC_HIP((launch_cgemm<T>(p, st)));
  return QCHEFF_OK;
}

// ------------------------------------------------------- recursive LU solve
//
// Solve q R = p for the chunk's augmented systems [q | p] in place (R lands in
// the right half).  factor(k0, k1) factors columns [k0, k1) over rows [k0, d)
// after every update from the columns left of k0 has been applied to them.
struct LuCtx {
  double2* aug;
  int* piv;
  int64_t d, ld, stride, nb;
  hipStream_t st;
  int panel_nb;     // leaf width of the factorization
  int panel_rows;   // register panel: rows per item it can hold (0: global-memory panel)
  // where the backward solve's leaves also place R (at most one of the two)
  const LuPlace<float2>* place32 = nullptr;
  const LuPlace<double2>* place64 = nullptr;
};

int lu_gemm_update(const LuCtx& c, int64_t r0, int64_t r1, int64_t c0, int64_t c1, int64_t k0, int64_t k1) {
  // A[r0:r1, c0:c1] -= A[r0:r1, k0:k1] * A[k0:k1, c0:c1]
  if (r1 <= r0 || c1 <= c0 || k1 <= k0) return QCHEFF_OK;
  // narrow updates (a 32-row leaf block, a 16-column panel) and short ones
  // (K <= 64, bound by reading and writing C) take the small tile
  const int cfg = (r1 - r0 <= 48 || c1 - c0 <= 48 || k1 - k0 <= 64) ? 1 : rule_cfg(c.d);
  auto p = gemm_params<double>(int(r1 - r0), int(c1 - c0), int(k1 - k0), int(c.nb), cfg);
  p.A = c.aug + r0 * c.ld + k0; p.lda = c.ld; p.sA = c.stride;
  p.B = c.aug + k0 * c.ld + c0; p.ldb = c.ld; p.sB = c.stride;
  p.C = c.aug + r0 * c.ld + c0; p.ldc = c.ld; p.sC = c.stride;
  p.alpha = -1.0; p.beta = 1.0;
  QC_HIP((launch_cgemm<double>(p, c.st)));
  return QCHEFF_OK;
}

int lu_pivots(const LuCtx& c, int64_t k0, int64_t k1, int64_t c0, int64_t c1) {
  if (c1 <= c0 || k1 <= k0) return QCHEFF_OK;
  hipLaunchKernelGGL(lu_pivots_kernel, dim3(nblocks(c1 - c0, 256), unsigned(c.nb)), dim3(256), 0, c.st, c.aug, c.ld,
                     c.stride, int(c.d), int(k0), int(k1), int(c0), int(c1), c.piv);
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

int64_t split_point(int64_t r0, int64_t r1, int64_t unit) {
  const int64_t half = (r1 - r0) / 2;
  return r0 + std::max<int64_t>(unit, (half + unit - 1) / unit * unit);
}

// X <- L^{-1} X, L unit lower on rows/cols [r0, r1), X = A[r0:r1, c0:c1]
int trsm_lower(const LuCtx& c, int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
  if (r1 - r0 <= kTrsmNb) {
    const dim3 grid(nblocks(c1 - c0, 256), unsigned(c.nb));
    if (r1 - r0 == kTrsmNb)
      hipLaunchKernelGGL(trsm_lower_unit_kernel, grid, dim3(256), 0, c.st, c.aug, c.ld, c.stride, int(r0), int(c0),
                         int(c1));
    else
      hipLaunchKernelGGL(trsm_lower_unit_ragged_kernel, grid, dim3(256), 0, c.st, c.aug, c.ld, c.stride, int(r0),
                         int(r1), int(c0), int(c1));
    QC_HIP(hipGetLastError());
    return QCHEFF_OK;
  }
  const int64_t h = split_point(r0, r1, kTrsmNb);
  int r;
  if ((r = trsm_lower(c, r0, h, c0, c1))) return r;
  if ((r = lu_gemm_update(c, h, r1, c0, c1, r0, h))) return r;
  return trsm_lower(c, h, r1, c0, c1);
}

// X <- U^{-1} X, U upper on rows/cols [r0, r1), X = A[r0:r1, c0:c1]
int trsm_upper(const LuCtx& c, int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
  if (r1 - r0 <= kTrsmNb) {
    const dim3 grid(nblocks(c1 - c0, 256), unsigned(c.nb));
    auto leaf = [&](auto pl) {
      using O = std::remove_pointer_t<decltype(pl.u0)>;
      if (r1 - r0 == kTrsmNb)
        hipLaunchKernelGGL(trsm_upper_kernel<O>, grid, dim3(256), 0, c.st, c.aug, c.ld, c.stride, int(r0), int(c0),
                           int(c1), pl);
      else
        hipLaunchKernelGGL(trsm_upper_ragged_kernel<O>, grid, dim3(256), 0, c.st, c.aug, c.ld, c.stride, int(r0),
                           int(r1), int(c0), int(c1), pl);
    };
    if (c.place32)
      leaf(*c.place32);
    else if (c.place64)
      leaf(*c.place64);
    else
      leaf(LuPlace<void>{nullptr, nullptr, nullptr, 0});
    QC_HIP(hipGetLastError());
    return QCHEFF_OK;
  }
  const int64_t h = split_point(r0, r1, kTrsmNb);
  int r;
  if ((r = trsm_upper(c, h, r1, c0, c1))) return r;
  if ((r = lu_gemm_update(c, r0, h, c0, c1, h, r1))) return r;
  return trsm_upper(c, r0, h, c0, c1);
}

int lu_panel(const LuCtx& c, int64_t k0, int64_t k1) {
  const unsigned g = unsigned(c.nb);
  const int d = int(c.d);
  if (c.panel_rows == 1024)
    hipLaunchKernelGGL((lu_panel_reg_kernel<16>), dim3(g), dim3(1024), 0, c.st, c.aug, c.ld, c.stride, d, int(k0),
                       int(k1), c.piv);
  else
    hipLaunchKernelGGL(lu_panel_kernel, dim3(g), dim3(256), 0, c.st, c.aug, c.ld, c.stride, d, int(k0), int(k1),
                       c.piv);
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

// Factors columns [k0, k1) and applies their L (row interchanges, forward
// solve) to the columns [k1, cend) as well.  Called with cend = k1 inside the
// left half; along the right edge of the recursion (k1 = d) cend = 2d carries the
// right-hand sides p, so their forward solve rides in the same launches as the
// factorization's own updates instead of a recursion of its own.
int lu_factor(const LuCtx& c, int64_t k0, int64_t k1, int64_t cend) {
  int r;
  if (k1 - k0 <= c.panel_nb) {
    if ((r = lu_panel(c, k0, k1))) return r;
    if (cend <= k1) return QCHEFF_OK;
    if ((r = lu_pivots(c, k0, k1, k1, cend))) return r;
    return trsm_lower(c, k0, k1, k1, cend);
  }
  const int64_t km = split_point(k0, k1, c.panel_nb);
  if ((r = lu_factor(c, k0, km, km))) return r;
  if ((r = lu_pivots(c, k0, km, km, cend))) return r;          // left pivots on the right part
  if ((r = trsm_lower(c, k0, km, km, cend))) return r;         // U12 = L11^{-1} A12
  if ((r = lu_gemm_update(c, km, c.d, km, cend, k0, km))) return r;  // A22 -= L21 U12
  if ((r = lu_factor(c, km, k1, cend))) return r;
  return lu_pivots(c, km, k1, k0, km);                       // right pivots on the left half's L
}

int lu_solve(double2* aug, int* piv, int64_t d, int64_t nb, hipStream_t st,
             const LuPlace<float2>* place32 = nullptr, const LuPlace<double2>* place64 = nullptr) {
  LuCtx c{aug, piv, d, 2 * d, 2 * d * d, nb, st, 32, 0, place32, place64};
  if (d <= 1024) { c.panel_nb = 16; c.panel_rows = 1024; }
  int r;
  if ((r = lu_factor(c, 0, d, 2 * d))) return r;             // P, L^{-1} on p along the way
  return trsm_upper(c, 0, d, d, 2 * d);                      // R = U^{-1} Y
}

// Side streams of one exponential call on the current device (default
// priority), the events that fork work onto them and join it back, and pinned
// host buffers for the squaring counts.  A call leases one set from a per-device
// pool for its duration and hands it back at the end, so concurrent calls from
// several host threads never share a set; sets are created on demand and kept
// for the life of the process.  A set goes back with work still queued on its
// streams, which only orders the next user's work behind it; every copy into
// its pinned buffers has been waited on by then.
struct SideStreams {
  static constexpr int kCount = 4;
  hipStream_t stream[kCount] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kCount] = {};
  hipEvent_t counts = nullptr;     // the squaring counts have reached the host
  int* pinned = nullptr;           // host copies of the squaring counts
  size_t pinned_n = 0;
};

struct SideLease {
  SideStreams* s = nullptr;
  int dev = 0;
  SideLease() = default;
  SideLease(const SideLease&) = delete;
  SideLease& operator=(const SideLease&) = delete;
  ~SideLease();
};

std::mutex g_side_mu;
std::map<int, std::vector<SideStreams*>> g_side_free;

SideLease::~SideLease() {
  if (!s) return;
  std::lock_guard<std::mutex> lk(g_side_mu);
  g_side_free[dev].push_back(s);
}

int lease_side(SideLease& out) {
  if (out.s) return QCHEFF_OK;
  QC_HIP(hipGetDevice(&out.dev));
  {
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto& v = g_side_free[out.dev];
    if (!v.empty()) {
      out.s = v.back();
      v.pop_back();
      return QCHEFF_OK;
    }
  }
  auto* s = new SideStreams{};
  for (int k = 0; k < SideStreams::kCount; ++k) {
    QC_HIP(hipStreamCreateWithFlags(&s->stream[k], hipStreamNonBlocking));
    QC_HIP(hipEventCreateWithFlags(&s->join[k], hipEventDisableTiming));
  }
  QC_HIP(hipEventCreateWithFlags(&s->counts, hipEventDisableTiming));
  QC_HIP(hipEventCreateWithFlags(&s->fork, hipEventDisableTiming));
  out.s = s;
  return QCHEFF_OK;
}

// A pinned host buffer of at least n ints (grown on demand: every copy into the
// old one has been waited on before the set went back to the pool).
int pinned_counts(SideStreams* s, size_t n, int** out) {
  if (s->pinned_n < n) {
    if (s->pinned) QC_HIP(hipHostFree(s->pinned));
    s->pinned = nullptr;
    s->pinned_n = 0;
    QC_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->pinned), std::max<size_t>(n, 1024) * sizeof(int),
                         hipHostMallocDefault));
    s->pinned_n = std::max<size_t>(n, 1024);
  }
  *out = s->pinned;
  return QCHEFF_OK;
}

// One chunk of one dimension group in a round of the exponential: its input
// and outputs (U, or U64 with the unitary refinement: an FP64 destination of
// the refined result, U then null) and its carved workspace.
template <typename T> struct ExpmChunk {
  const typename Cx<T>::t* omega;
  typename Cx<T>::t* U;
  double2* U64;
  int32_t* s_out;
  int64_t nb, d;
  ExpmWs<T> w;
};

// One product stage over the round's groups: a single group takes the
// per-launch kernel (with the timing record), several the grouped kernel, a
// workgroup per tile slot (eight times the busiest XCD's slot count).
template <typename T, int CFG, int MODE = 0>
hipError_t launch_grouped_cfg(const GemmGroups<T>& gg, hipStream_t st) {
  using G = GemmTile<T, CFG>;
  auto kern = cgemm_grouped_kernel<T, G::BM, G::BN, G::BK, G::WM, G::WN, G::NT, G::WPE, MODE>;
  hipLaunchKernelGGL(kern, dim3(unsigned(kXcds * gg.per_xcd)), dim3(G::NT), 0, st, gg);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stage(GemmParams<T>* p, int G, hipStream_t st, const int64_t* active = nullptr) {
  if (G == 1) return launch_cgemm<T>(p[0], st, active ? active[0] : -1);
  if (split_bf16_cfg(p[0].cfg)) {   // split-BF16 tiles (FP32 only): per group
    for (int g = 0; g < G; ++g)
      if (hipError_t e = launch_cgemm<T>(p[g], st, active ? active[g] : -1)) return e;
    return hipSuccess;
  }
  GemmGroups<T> gg{};
  gg.G = G;
  double flops = 0.0, bytes = 0.0;
  int64_t xslots[kXcds] = {};
  for (int g = 0; g < G; ++g) {
    gg.p[g] = p[g];
    const bool empty = p[g].M <= 0 || p[g].N <= 0 || p[g].batch <= 0;
    const int64_t tiles = empty ? 0
                        : p[g].herm ? int64_t(p[g].tiles_m) * (p[g].tiles_m + 1) / 2
                                    : int64_t(p[g].tiles_m) * p[g].tiles_n;
    // the group's items split evenly over the XCDs
    for (int x = 0; x < kXcds; ++x) {
      const int64_t i0 = empty ? 0 : int64_t(p[g].batch) * x / kXcds;
      const int64_t i1 = empty ? 0 : int64_t(p[g].batch) * (x + 1) / kXcds;
      gg.item0[x][g] = int(i0);
      gg.base[x][g] = int(xslots[x]);
      xslots[x] += (i1 - i0) * tiles;
    }
    const double outs = p[g].herm ? double(p[g].M) * (p[g].M + 1) / 2 : double(p[g].M) * p[g].N;
    const double act = double(active ? active[g] : p[g].batch);
    flops += 8.0 * outs * double(p[g].K) * act;
    bytes += (double(p[g].M) * p[g].K + double(p[g].K) * p[g].N + double(p[g].M) * p[g].N) *
             sizeof(typename Cx<T>::t) * act;
  }
  int64_t most = 0;
  for (int x = 0; x < kXcds; ++x) {
    gg.base[x][G] = int(xslots[x]);
    most = std::max(most, xslots[x]);
  }
  if (most == 0) return hipSuccess;
  if (most * kXcds > 0x7fffffff) return hipErrorInvalidValue;
  gg.per_xcd = int(most);
  LaunchTimer tm;
  tm.begin(st);
  hipError_t e;
  if constexpr (sizeof(T) == 8) {
    if (p[0].mode == 1) {   // FP64 products of complex64 operands: cfg 0 or 1
      for (int g = 0; g < G; ++g)
        if (p[g].mode != 1 || p[g].cfg != p[0].cfg || !p[g].a32 || p[g].M != p[g].N || p[g].N != p[g].K)
          return hipErrorInvalidValue;
      e = p[0].cfg == 1 ? launch_grouped_cfg<T, 1, 1>(gg, st)
        : p[0].cfg == 0 ? launch_grouped_cfg<T, 0, 1>(gg, st)
                        : hipErrorInvalidValue;
      if (tm.on) tm.end(st, KERNEL_GEMM_F64, flops, bytes);
      return e;
    }
  }
  e = p[0].cfg == 1   ? launch_grouped_cfg<T, 1>(gg, st)
    : p[0].cfg == 4 ? launch_grouped_cfg<T, 4>(gg, st)
                    : launch_grouped_cfg<T, 0>(gg, st);
  if (tm.on) tm.end(st, sizeof(T) == 8 ? KERNEL_GEMM_F64 : KERNEL_GEMM_F32, flops, bytes);
  return e;
}

// Product parameters for one chunk: out = A B (+ sum_i xc[i] X_i + gamma I).
template <typename T>
GemmParams<T> chunk_product(int cfg, int herm, typename Cx<T>::t* out, const typename Cx<T>::t* A,
                            const typename Cx<T>::t* B, int64_t d, int64_t nb, int nx = 0,
                            const typename Cx<T>::t* const* X = nullptr, const T* xc = nullptr, T gamma = T(0)) {
  auto p = gemm_params<T>(int(d), int(d), int(d), int(nb), cfg);
  p.herm = herm;
  const int64_t dd = d * d;
  p.A = A; p.lda = d; p.sA = dd;
  p.B = B; p.ldb = d; p.sB = dd;
  p.C = out; p.ldc = d; p.sC = dd;
  p.nx = nx;
  for (int i = 0; i < nx; ++i) { p.X[i] = X[i]; p.xc[i] = xc[i]; }
  p.gamma = gamma;
  return p;
}

// The product tile of a round: the split-BF16 kernel, or the configuration the
// tuner picked for the group with the most product work.
template <typename T>
int round_cfg(ExpmChunk<T>* ch, int G, bool bf16x3, bool skew, hipStream_t st, int* cfg) {
  if (bf16x3) {
    *cfg = bf16x3_cfg();
    return QCHEFF_OK;
  }
  int gmax = 0;
  for (int g = 1; g < G; ++g)
    if (double(ch[g].d) * ch[g].d * ch[g].d * ch[g].nb > double(ch[gmax].d) * ch[gmax].d * ch[gmax].d * ch[gmax].nb)
      gmax = g;
  // the tuner times on the scaled A of that group, into its W (free before the products)
  return square_cfg<T>(ch[gmax].d, ch[gmax].nb, ch[gmax].w.X[0], ch[gmax].w.X[4], skew, st, cfg);
}

// The exponential of a round (a chunk of each of G dimension groups; G = 1 for
// qcheff_expm_batched) runs in three stages:
//   A  per group the norm, the scaling and the squaring counts (copied to the
//      host unless a bound is given), then the Pade products and the augmented
//      system, each product stage one launch over all groups;
//   B  per group the FP64 solve and the placing of its result (several groups'
//      solves side by side on the side streams);
//   C  the squarings (one launch over all groups per step), the refinement and
//      the phase.
// The tile of the products is chosen in the first round's stage A (cfg < 0 on
// entry: after the scaling, by round_cfg) and kept for the later ones, so that
// an item's rounding does not depend on which round it falls in.
template <typename T> struct RoundState {
  using C2 = typename Cx<T>::t;
  const double2* mu[kMaxGroups] = {};
  C2* Ubuf[kMaxGroups] = {};
  C2* sq0[kMaxGroups] = {};
  C2* sq1[kMaxGroups] = {};
  int* s_host[kMaxGroups] = {};   // pinned copies of the squaring counts (bound < 0)
  hipEvent_t s_ready = nullptr;   // recorded after those copies
};

template <typename T>
int expm_stage_a(ExpmChunk<T>* ch, int G, RoundState<T>& rs, int* cfg_io, bool bf16x3, bool skew, int bound,
                 bool refine, hipStream_t st) {
  using C2 = typename Cx<T>::t;
  double b[14];
  pade_coefficients(13, b);
  const T c[14] = {T(b[0]), T(b[1]), T(b[2]), T(b[3]), T(b[4]), T(b[5]), T(b[6]),
                   T(b[7]), T(b[8]), T(b[9]), T(b[10]), T(b[11]), T(b[12]), T(b[13])};
  for (int g = 0; g < G; ++g) {
    ExpmChunk<T>& k = ch[g];
    ExpmWs<T>& w = k.w;
    const int64_t d = k.d, nb = k.nb, dd = d * d;
    rs.Ubuf[g] = k.U ? k.U : reinterpret_cast<C2*>(k.U64);   // the chunk's destination, as scratch of its own type
    // norms and smax start at zero (a fill kernel, not a memset)
    hipLaunchKernelGGL(fill_u32_kernel, dim3(nblocks(nb * 2, 256)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(w.norms), nb * 2, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(w.smax), int64_t(1),
                       0u);
    QC_HIP(hipGetLastError());
    // Trace reduction in FP64 only: exp(Omega) = e^mu exp(Omega - mu I), mu = tr(Omega) / d.
    // It centres the spectrum, which for a drift-dominated generator halves the
    // norm (one squaring less) but moves the low-energy end, where such a system's
    // states live, from the middle of the scaled spectrum (where the Pade
    // approximant is most accurate) to its edge; in FP32 that costs more accuracy
    // in those states than the saved squaring wins.
    if (sizeof(T) == 8) {
      hipLaunchKernelGGL(trace_mean_kernel<C2>, dim3(unsigned(nb)), dim3(256), 0, st, k.omega, int(d), w.mu);
      rs.mu[g] = w.mu;
    }
    {
      // partial column sums per 128-row tile go to the augmented-system buffer,
      // which is not in use before the Pade products
      const unsigned tiles = nblocks(d, kNormRows);
      double* partial = reinterpret_cast<double*>(w.aug);
      hipLaunchKernelGGL(norm1_partial_kernel<C2>, dim3(nblocks(d, 64), tiles, unsigned(nb)), dim3(256), 0, st,
                         k.omega, int(d), rs.mu[g], partial);
      hipLaunchKernelGGL(norm1_finish_kernel, dim3(unsigned(nb)), dim3(256), 0, st, partial, int(d), int(tiles),
                         w.norms);
    }
    QC_HIP(hipGetLastError());
    const unsigned sblocks = unsigned(std::min<int64_t>(nblocks(dd, 256), 1024));
    hipLaunchKernelGGL(scale_kernel<C2>, dim3(sblocks, unsigned(nb)), dim3(256), 0, st, k.omega, w.X[0], int(d),
                       rs.mu[g], w.norms, kTheta13, bound, w.s_ws, k.s_out, w.smax);
    QC_HIP(hipGetLastError());
    // Without a bound the host reads the squaring counts back to size the
    // squaring launches (stage C waits for them, long after they are ready)
    if (bound < 0) QC_HIP(hipMemcpyAsync(rs.s_host[g], w.s_ws, size_t(nb) * sizeof(int), hipMemcpyDeviceToHost, st));
  }
  if (bound < 0) QC_HIP(hipEventRecord(rs.s_ready, st));
  if (*cfg_io < 0)   // a split-BF16 tile, or the tuned FP32 / FP64 one
    if (int r = round_cfg<T>(ch, G, bf16x3, skew, st, cfg_io)) return r;
  const int cfg = *cfg_io;
  // For skew-Hermitian A every even power, W and V are Hermitian (and A W
  // skew-Hermitian): only half of each of those products is formed.
  const int h = skew ? 1 : 0;
  GemmParams<T> p[kMaxGroups];
  for (int g = 0; g < G; ++g) { auto& w = ch[g].w; p[g] = chunk_product<T>(cfg, h, w.X[1], w.X[0], w.X[0], ch[g].d, ch[g].nb); }
  QC_HIP(launch_stage<T>(p, G, st));   // A^2
  for (int g = 0; g < G; ++g) { auto& w = ch[g].w; p[g] = chunk_product<T>(cfg, h, w.X[2], w.X[1], w.X[1], ch[g].d, ch[g].nb); }
  QC_HIP(launch_stage<T>(p, G, st));   // A^4
  for (int g = 0; g < G; ++g) { auto& w = ch[g].w; p[g] = chunk_product<T>(cfg, h, w.X[3], w.X[2], w.X[1], ch[g].d, ch[g].nb); }
  QC_HIP(launch_stage<T>(p, G, st));   // A^6
  // W = A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I   (U = A W)
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  // The inner combinations go to buffers that are free at this point: the
  // chunk's U (its input was consumed by the scaling; with an FP64 destination,
  // the first half of that) and W.  V is formed first (from W), then W (from U)
  // overwrites its own buffer.  The outer terms are added by the epilogues.
  for (int g = 0; g < G; ++g) {
    auto& w = ch[g].w;
    const int64_t n = ch[g].nb * ch[g].d * ch[g].d;
    hipLaunchKernelGGL((pade_inner_kernel<C2, T>), dim3(unsigned(std::min<int64_t>(nblocks(n, 256), 8192))),
                       dim3(256), 0, st, w.X[3], w.X[2], w.X[1], n, c[13], c[11], c[9], c[12], c[10], c[8], rs.Ubuf[g],
                       w.X[4]);
  }
  QC_HIP(hipGetLastError());
  const T xv[3] = {c[6], c[4], c[2]};
  const T xw[3] = {c[7], c[5], c[3]};
  for (int g = 0; g < G; ++g) {
    auto& w = ch[g].w;
    const C2* Xs[3] = {w.X[3], w.X[2], w.X[1]};
    p[g] = chunk_product<T>(cfg, h, w.X[5], w.X[3], w.X[4], ch[g].d, ch[g].nb, 3, Xs, xv, c[0]);
  }
  QC_HIP(launch_stage<T>(p, G, st));   // V
  for (int g = 0; g < G; ++g) {
    auto& w = ch[g].w;
    const C2* Xs[3] = {w.X[3], w.X[2], w.X[1]};
    p[g] = chunk_product<T>(cfg, h, w.X[4], w.X[3], rs.Ubuf[g], ch[g].d, ch[g].nb, 3, Xs, xw, c[1]);
  }
  QC_HIP(launch_stage<T>(p, G, st));   // W
  // [q | p] = [V - A W | V + A W] in FP64
  for (int g = 0; g < G; ++g) {
    auto& w = ch[g].w;
    const int64_t d = ch[g].d, dd = d * d;
    p[g] = chunk_product<T>(cfg, -h, w.X[5], w.X[0], w.X[4], d, ch[g].nb);
    p[g].X[0] = w.X[5];
    p[g].epi = EPI_AUG;
    p[g].aug = w.aug; p[g].ld_aug = 2 * d; p[g].s_aug = 2 * dd; p[g].aug_off = d;
  }
  QC_HIP(launch_stage<T>(p, G, st));
  // The squarings ping-pong between the chunk's U and A; with the unitary
  // refinement they run in W and V instead (the refinement reads the last one
  // and writes U).  W and V are free once the augmented system is formed.
  for (int g = 0; g < G; ++g) {
    rs.sq0[g] = refine ? ch[g].w.X[4] : ch[g].U;
    rs.sq1[g] = refine ? ch[g].w.X[5] : ch[g].w.X[0];
  }
  return QCHEFF_OK;
}

// Stage B on stream sb.  Several groups' solves run side by side on the side
// streams, forked from and joined back into sb through events (which graph
// capture records as dependencies): a solve is a chain of many small dependent
// launches, and the groups' chains fill each other's idle time.
template <typename T>
int expm_stage_b(ExpmChunk<T>* ch, int G, RoundState<T>& rs, SideStreams* set, hipStream_t sb) {
  using C2 = typename Cx<T>::t;
  SideStreams* side = G > 1 ? set : nullptr;
  if (side) QC_HIP(hipEventRecord(side->fork, sb));
  for (int g = 0; g < G; ++g) {
    auto& w = ch[g].w;
    const int64_t d = ch[g].d, dd = d * d;
    hipStream_t sg = sb;
    if (side) {
      sg = side->stream[g % SideStreams::kCount];
      QC_HIP(hipStreamWaitEvent(sg, side->fork, 0));
    }
    // the solve's last leaves place R where the squarings start
    const LuPlace<C2> pl{w.s_ws, rs.sq0[g], rs.sq1[g], int(d)};
    int r;
    if constexpr (std::is_same_v<C2, float2>)
      r = lu_solve(w.aug, w.piv, d, ch[g].nb, sg, &pl, nullptr);
    else
      r = lu_solve(w.aug, w.piv, d, ch[g].nb, sg, nullptr, &pl);
    if (r) return r;
  }
  if (side) {
    for (int k = 0; k < std::min(G, SideStreams::kCount); ++k) {
      QC_HIP(hipEventRecord(side->join[k], side->stream[k]));
      QC_HIP(hipStreamWaitEvent(sb, side->join[k], 0));
    }
  }
  return QCHEFF_OK;
}

// Stage C: with a bound exactly `bound` squaring passes are enqueued (an item
// leaves the passes once its own count is done) and nothing waits; without, the
// host takes the counts stage A copied.
template <typename T>
int expm_stage_c(ExpmChunk<T>* ch, int G, RoundState<T>& rs, int cfg, int bound, bool refine, hipStream_t st) {
  using C2 = typename Cx<T>::t;
  if (bound < 0) QC_HIP(hipEventSynchronize(rs.s_ready));
  int smax = 0;
  for (int g = 0; g < G; ++g)
    for (int64_t i = 0; i < ch[g].nb; ++i) smax = std::max(smax, bound < 0 ? rs.s_host[g][i] : bound);
  GemmParams<T> p[kMaxGroups];
  for (int step = 0; step < smax; ++step) {
    int64_t active[kMaxGroups];
    for (int g = 0; g < G; ++g) {
      const int64_t d = ch[g].d, dd = d * d;
      active[g] = bound >= 0 ? ch[g].nb
                             : std::count_if(rs.s_host[g], rs.s_host[g] + ch[g].nb, [step](int s) { return s > step; });
      p[g] = gemm_params<T>(int(d), int(d), int(d), int(ch[g].nb), cfg);
      p[g].lda = d; p[g].ldb = d; p[g].ldc = d;
      p[g].sA = dd; p[g].sB = dd; p[g].sC = dd;
      p[g].sq = 1; p[g].sq_s = ch[g].w.s_ws; p[g].sq_step = step; p[g].sq_p0 = rs.sq0[g]; p[g].sq_p1 = rs.sq1[g];
    }
    QC_HIP(launch_stage<T>(p, G, st, active));
  }
  if constexpr (sizeof(T) == 4) {
    if (refine) {
      // One Newton step of the polar decomposition: E = I - R R^dag for the FP32
      // result R (in sq0), then U = R + (1/2) E R.  E is formed on the FP64
      // matrix cores straight from R's complex64 values (their products are exact
      // in FP64, so the sum carries FP64 accuracy) and written in complex64,
      // enough for the small correction product; it takes the space of A^4.
      GemmParams<double> pd[kMaxGroups];
      int64_t dmax = 0;
      for (int g = 0; g < G; ++g) dmax = std::max(dmax, ch[g].d);
      for (int g = 0; g < G; ++g) {
        auto& w = ch[g].w;
        const int64_t d = ch[g].d, dd = d * d;
        pd[g] = gemm_params<double>(int(d), int(d), int(d), int(ch[g].nb), rule_cfg(dmax));
        pd[g].mode = 1;
        pd[g].a32 = reinterpret_cast<const float2*>(rs.sq0[g]); pd[g].ld32 = d; pd[g].s32 = dd;
        pd[g].lda = d; pd[g].ldb = d;
        pd[g].epi = EPI_C32;
        pd[g].c32 = reinterpret_cast<float2*>(w.X[2]);
        pd[g].C = reinterpret_cast<double2*>(w.X[2]); pd[g].ldc = d; pd[g].sC = dd;   // not written
        pd[g].alpha = -1.0; pd[g].gamma = 1.0; pd[g].herm = 1;
      }
      QC_HIP(launch_stage<double>(pd, G, st));
      for (int g = 0; g < G; ++g) {
        auto& w = ch[g].w;
        const int64_t d = ch[g].d, dd = d * d;
        p[g] = chunk_product<T>(cfg, 0, ch[g].U64 ? rs.sq0[g] : ch[g].U, w.X[2], rs.sq0[g], d, ch[g].nb);
        p[g].alpha = T(0.5);
        p[g].nx = 1; p[g].X[0] = rs.sq0[g]; p[g].xc[0] = T(1);
        if (ch[g].U64) {   // R + (1/2) E R formed and kept in FP64: no final rounding to FP32
          p[g].epi = EPI_OUT64;
          p[g].aug = ch[g].U64; p[g].ld_aug = d; p[g].s_aug = dd;
        }
      }
      QC_HIP(launch_stage<T>(p, G, st));
    }
  }
  for (int g = 0; g < G; ++g) {
    if (!rs.mu[g]) continue;
    const int64_t dd = ch[g].d * ch[g].d;
    const unsigned sblocks = unsigned(std::min<int64_t>(nblocks(dd, 256), 1024));
    hipLaunchKernelGGL(phase_kernel<C2>, dim3(sblocks, unsigned(ch[g].nb)), dim3(256), 0, st, ch[g].U, dd, rs.mu[g]);
    QC_HIP(hipGetLastError());
  }
  return QCHEFF_OK;
}

// Host-side state of a round: the pinned count buffer and its event, from the
// call's set of side streams.
template <typename T>
int round_state(ExpmChunk<T>* ch, int G, int bound, SideStreams* side, RoundState<T>& rs) {
  if (bound >= 0) return QCHEFF_OK;
  size_t total = 0;
  for (int g = 0; g < G; ++g) total += size_t(ch[g].nb);
  int* buf = nullptr;
  if (int r = pinned_counts(side, total, &buf)) return r;
  for (int g = 0; g < G; ++g) {
    rs.s_host[g] = buf;
    buf += ch[g].nb;
  }
  rs.s_ready = side->counts;
  return QCHEFF_OK;
}

// One round, the three stages in order on `st`.
template <typename T>
int expm_round(ExpmChunk<T>* ch, int G, int* cfg_io, bool bf16x3, bool skew, int bound, bool refine,
               SideStreams* side, hipStream_t st) {
  RoundState<T> rs;
  if (int r = round_state<T>(ch, G, bound, side, rs)) return r;
  if (int r = expm_stage_a<T>(ch, G, rs, cfg_io, bf16x3, skew, bound, refine, st)) return r;
  if (int r = expm_stage_b<T>(ch, G, rs, side, st)) return r;
  return expm_stage_c<T>(ch, G, rs, *cfg_io, bound, refine, st);
}

template <typename T>
int run_expm(const void* omega, int64_t batch, int64_t d, void* U, int32_t* s_out, void* ws, size_t ws_bytes,
             int dtype, bool skew, int bound, bool bf16x3, bool refine, bool out64, hipStream_t st) {
  using C2 = typename Cx<T>::t;
  if (d <= kSmallD) {
    // one workgroup per item, everything in LDS; no workspace and no host sync
    const unsigned grid = unsigned(std::min<int64_t>(batch, 256 * 8));
    hipLaunchKernelGGL(expm_small_kernel<T>, dim3(grid), dim3(256), 0, st, static_cast<const C2*>(omega),
                       out64 ? nullptr : static_cast<C2*>(U), out64 ? static_cast<double2*>(U) : nullptr, s_out,
                       int(d), int(batch), kTheta13, refine ? 1 : 0);
    QC_HIP(hipGetLastError());
    return QCHEFF_OK;
  }
  const int64_t dd = d * d;
  SideLease lease;
  if (int r = lease_side(lease)) return r;
  auto chunk_at = [&](ExpmChunk<T>& c, int64_t b0, int64_t nb) {
    c.nb = nb;
    c.d = d;
    c.omega = static_cast<const C2*>(omega) + b0 * dd;
    c.U = out64 ? nullptr : static_cast<C2*>(U) + b0 * dd;
    c.U64 = out64 ? static_cast<double2*>(U) + b0 * dd : nullptr;
    c.s_out = s_out ? s_out + b0 : nullptr;
  };
  int cfg = -1;
  // a chunk's items ride on the grid's y (or z) dimension
  const int64_t chunk = std::min<int64_t>(expm_chunk(ws_bytes, batch, d, dtype), 65535);
  ExpmChunk<T> ch{};
  if (!carve_expm<T>(ws, ws_bytes, chunk, d, ch.w)) return fail(QCHEFF_EWORKSPACE, "workspace carving failed");
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    chunk_at(ch, b0, std::min(chunk, batch - b0));
    if (int r = expm_round<T>(&ch, 1, &cfg, bf16x3, skew, bound, refine, lease.s, st)) return r;
  }
  return QCHEFF_OK;
}

// qcheff_expm_grouped: the groups with d <= 32 through the fused kernel, the
// others in rounds of expm_round.  The number of rounds R is the smallest for
// which every group's slice (its batch / R, rounded up) fits the workspace
// together with the others'.
template <typename T>
int run_expm_grouped(int G, const void* const* omega, const int64_t* batch, const int64_t* d, void* const* U,
                     int32_t* const* s_out, void* ws, size_t ws_bytes, int dtype, bool skew, int bound, bool bf16x3,
                     bool refine, bool out64, hipStream_t st) {
  using C2 = typename Cx<T>::t;
  int big[kMaxGroups];
  int nbig = 0;
  int64_t most = 0;
  for (int g = 0; g < G; ++g) {
    if (batch[g] == 0) continue;
    if (d[g] <= kSmallD) {
      if (int r = run_expm<T>(omega[g], batch[g], d[g], U[g], s_out ? s_out[g] : nullptr, nullptr, 0, dtype, skew,
                              bound, bf16x3, refine, out64, st))
        return r;
    } else {
      big[nbig++] = g;
      most = std::max(most, batch[g]);
    }
  }
  if (nbig == 0) return QCHEFF_OK;
  auto slice = [&](int g, int64_t R) { return std::min<int64_t>((batch[g] + R - 1) / R, 65535); };
  auto need = [&](int64_t R) {
    size_t n = 0;
    for (int k = 0; k < nbig; ++k) n += expm_ws_bytes(slice(big[k], R), d[big[k]], dtype);
    return n;
  };
  int64_t R = 1;
  while (R < most && need(R) > ws_bytes) {
    // shrink geometrically, then settle on the smallest R that fits
    const int64_t next = std::min(most, R * 2);
    if (need(next) > ws_bytes) { R = next; continue; }
    int64_t lo = R + 1, hi = next;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (need(mid) <= ws_bytes) hi = mid; else lo = mid + 1;
    }
    R = lo;
    break;
  }
  if (need(R) > ws_bytes) return fail(QCHEFF_EWORKSPACE, "qcheff_expm_grouped: workspace carving failed");
  ExpmWs<T> w[kMaxGroups];
  int64_t chunk[kMaxGroups];
  {
    char* at = static_cast<char*>(ws);
    size_t left = ws_bytes;
    for (int k = 0; k < nbig; ++k) {
      const int g = big[k];
      chunk[k] = slice(g, R);
      const size_t n = expm_ws_bytes(chunk[k], d[g], dtype);
      if (n > left || !carve_expm<T>(at, n, chunk[k], d[g], w[k]))
        return fail(QCHEFF_EWORKSPACE, "qcheff_expm_grouped: workspace carving failed");
      at += n;
      left -= n;
    }
  }
  SideLease lease;
  if (int e = lease_side(lease)) return e;
  int cfg = -1;   // every group has items in the first round, which picks the tile
  for (int64_t r = 0;; ++r) {
    ExpmChunk<T> ch[kMaxGroups];
    int n = 0;
    for (int k = 0; k < nbig; ++k) {
      const int g = big[k];
      const int64_t b0 = r * chunk[k];
      if (b0 >= batch[g]) continue;
      const int64_t dd = d[g] * d[g];
      ExpmChunk<T>& c = ch[n++];
      c.nb = std::min(chunk[k], batch[g] - b0);
      c.d = d[g];
      c.omega = static_cast<const C2*>(omega[g]) + b0 * dd;
      c.U = out64 ? nullptr : static_cast<C2*>(U[g]) + b0 * dd;
      c.U64 = out64 ? static_cast<double2*>(U[g]) + b0 * dd : nullptr;
      c.s_out = (s_out && s_out[g]) ? s_out[g] + b0 : nullptr;
      c.w = w[k];
    }
    if (n == 0) break;
    if (int e = expm_round<T>(ch, n, &cfg, bf16x3, skew, bound, refine, lease.s, st)) return e;
  }
  return QCHEFF_OK;
}

// --------------------------------------------------------------------- NPAD
struct NpadWs {
  int* mark;
  NpadRot* rot;
  int* active;
  Best* part;
};

bool carve_npad(void* ws, size_t bytes, int64_t P, int64_t d, NpadWs& w) {
  Carver cv{static_cast<char*>(ws), bytes};
  w.mark = cv.take<int>(size_t(d) * 4);
  w.rot = cv.take<NpadRot>(size_t(std::max<int64_t>(P, 1)) * sizeof(NpadRot));
  w.active = cv.take<int>(size_t(std::max<int64_t>(P, 1)) * 4);
  w.part = cv.take<Best>(size_t((d + 3) / 4) * sizeof(Best));
  return w.mark && w.rot && w.active && w.part;
}

template <typename C2>
int run_npad_eliminate(C2* H, int64_t d, const int64_t* pairs, int64_t P, NpadWs& w, hipStream_t st) {
  if (P == 0) return QCHEFF_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(nblocks(d, 256)), dim3(256), 0, st, reinterpret_cast<uint32_t*>(w.mark), d,
                     0u);
  hipLaunchKernelGGL(npad_mark_kernel, dim3(nblocks(P, 256)), dim3(256), 0, st, pairs, P, d, w.mark);
  hipLaunchKernelGGL(npad_params_kernel<C2>, dim3(nblocks(P, 256)), dim3(256), 0, st, H, d, pairs, P, w.mark, w.rot,
                     w.active);
  QC_HIP(hipGetLastError());
  const unsigned gx = unsigned(std::min<int64_t>(nblocks(d, 256), 64));
  for (int64_t p0 = 0; p0 < P; p0 += 65535) {
    const unsigned np = unsigned(std::min<int64_t>(65535, P - p0));
    hipLaunchKernelGGL(npad_rows_kernel<C2>, dim3(gx, np), dim3(256), 0, st, H, d, pairs, p0, w.rot, w.active);
  }
  QC_HIP(hipGetLastError());
  if (P >= 64) {
    // threads over the pairs of a row; rows spread over grid y
    const unsigned gy = unsigned(std::min<int64_t>(d, 65535));
    hipLaunchKernelGGL((npad_cols_kernel<C2, true>), dim3(nblocks(P, 256), gy), dim3(256), 0, st, H, d, pairs, P,
                       int64_t(0), w.rot, w.active);
  } else {
    hipLaunchKernelGGL((npad_cols_kernel<C2, false>), dim3(gx, unsigned(P)), dim3(256), 0, st, H, d, pairs, P,
                       int64_t(0), w.rot, w.active);
  }
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

template <typename C2>
int run_npad_largest(const C2* H, int64_t d, int64_t* ij, double* mag, NpadWs& w, hipStream_t st) {
  const int64_t nb = (d + 3) / 4;
  hipLaunchKernelGGL(npad_largest_partial_kernel<C2>, dim3(unsigned(nb)), dim3(256), 0, st, H, d, w.part);
  hipLaunchKernelGGL(npad_largest_final_kernel, dim3(1), dim3(256), 0, st, w.part, nb, d, ij, mag);
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

// ---------------------------------------------------------------- propagate
// ------------------------------------------------------- state-only action
// sum_{k > m} x^k / k! (x >= 0), summed until the terms stop mattering.
double taylor_tail(double x, int m) {
  if (x <= 0.0) return 0.0;
  double term = std::exp((m + 1) * std::log(x) - std::lgamma(m + 2.0));
  double sum = 0.0;
  for (int k = m + 1; k < m + 2000; ++k) {
    sum += term;
    term *= x / double(k + 1);
    if (term <= 1e-17 * sum) break;
  }
  return sum;
}

// Degree m <= 55 and step count s of the truncated Taylor action for a generator
// whose shifted 2-norm is at most nu: the smallest m s with
// s * sum_{k>m} (nu/s)^k / k! <= tol (the truncation error of s steps, each
// exp of a matrix of 2-norm nu/s applied to a unit vector).  s * tail(nu/s) falls
// with s, so a bisection finds the smallest s for each m.
void action_params(double nu, double tol, int* m_out, int64_t* s_out) {
  int best_m = 0;
  int64_t best_s = 0;
  double best = 0.0;
  for (int m = 1; m <= 55; ++m) {
    auto ok = [&](int64_t s) { return double(s) * taylor_tail(nu / double(s), m) <= tol; };
    int64_t hi = 1;
    while (!ok(hi) && hi < (int64_t(1) << 40)) hi *= 2;
    if (!ok(hi)) continue;
    int64_t lo = hi / 2 + 1;
    if (hi == 1) lo = 1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (ok(mid)) hi = mid; else lo = mid + 1;
    }
    const double cost = double(m) * double(hi);
    if (best_m == 0 || cost < best) {
      best = cost;
      best_m = m;
      best_s = hi;
    }
  }
  *m_out = best_m;
  *s_out = best_s;
}

constexpr double kMaxActionTerms = double(1 << 24);   // products per interval

template <typename T>
int run_action(const void* Ov, int64_t M, int64_t d, void* x, void* traj, double tol, void* ws, size_t ws_bytes,
               bool skew, hipStream_t st) {
  using C2 = typename Cx<T>::t;
  const C2* Om = static_cast<const C2*>(Ov);
  const int64_t dd = d * d;
  Carver cv{static_cast<char*>(ws), ws_bytes};
  double2* X = cv.take<double2>(size_t(d) * 16);
  double2* Y = cv.take<double2>(size_t(d) * 16);
  double2* mu = cv.take<double2>(size_t(M) * 16);
  unsigned long long* norms = cv.take<unsigned long long>(size_t(M) * 16);
  const int nb = int((d + kActTile - 1) / kActTile);
  double2* P = cv.take<double2>(size_t(nb) * nb * kActTile * 16);
  const int mode = action_mode(d, skew);
  double2* F = static_cast<double2*>(x);
  double2* t = static_cast<double2*>(traj);
  if (t) QC_HIP(hipMemcpyAsync(t, F, size_t(d) * 16, hipMemcpyDeviceToDevice, st));
  if (M == 0) return QCHEFF_OK;
  if (tol <= 0.0) tol = sizeof(T) == 8 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(nblocks(4 * M, 256)), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(norms), 4 * M, 0u);
  hipLaunchKernelGGL(trace_mean_kernel<C2>, dim3(unsigned(M)), dim3(256), 0, st, Om, int(d), mu);
  // the tiled product already takes Omega as skew-Hermitian: then one row pass
  // gives both norms; otherwise columns and rows.  Items in slices of the
  // grid's y limit.
  for (int64_t b0 = 0; b0 < M; b0 += 65535) {
    const unsigned nbt = unsigned(std::min<int64_t>(65535, M - b0));
    if (mode == 1)
      hipLaunchKernelGGL(shifted_rownorm_kernel<C2>, dim3(nblocks(d, 4), nbt), dim3(256), 0, st, Om, int(d), b0, mu,
                         norms);
    else
      hipLaunchKernelGGL(shifted_norms_kernel<C2>, dim3(nblocks(d, 256), nbt, 2), dim3(256), 0, st, Om, int(d), b0,
                         mu, norms);
  }
  QC_HIP(hipGetLastError());
  // the host sizes every interval's launches from the shift and the norms
  std::vector<double2> mu_h(static_cast<size_t>(M));
  std::vector<unsigned long long> nb_h(static_cast<size_t>(2 * M));
  QC_HIP(hipMemcpyAsync(mu_h.data(), mu, size_t(M) * 16, hipMemcpyDeviceToHost, st));
  QC_HIP(hipMemcpyAsync(nb_h.data(), norms, size_t(2 * M) * 8, hipMemcpyDeviceToHost, st));
  QC_HIP(hipStreamSynchronize(st));
  const double qnan = std::nan("");
  for (int64_t n = 0; n < M; ++n) {
    double n1, ninf;
    std::memcpy(&n1, &nb_h[2 * n], 8);
    std::memcpy(&ninf, &nb_h[2 * n + 1], 8);
    if (mode == 1) n1 = ninf;                 // equal for a skew-Hermitian matrix
    const double nu = std::sqrt(n1 * ninf);   // ||.||_2 <= sqrt(||.||_1 ||.||_inf)
    const double2 m_n = mu_h[n];
    int m = 0;
    int64_t s = 1;
    if (!(nu <= 1.7976931348623157e308) || !std::isfinite(m_n.x) || !std::isfinite(m_n.y)) {
      m = -1;   // non-finite generator: the state becomes NaN
      flag_host_status(STATUS_NONFINITE);
    } else if (nu > 0.0) {
      action_params(nu, tol, &m, &s);
      if (m == 0 || double(m) * double(s) > kMaxActionTerms)
        return fail(QCHEFF_EUNSUPPORTED, "qcheff_propagate_action: generator norm too large for the Taylor action "
                                         "(use qcheff_expm_batched and qcheff_propagate)");
    }
    if (m <= 0) {
      const double2 eta = m < 0 ? make_double2(qnan, qnan)
                                : make_double2(std::exp(m_n.x) * std::cos(m_n.y), std::exp(m_n.x) * std::sin(m_n.y));
      hipLaunchKernelGGL(scale_state_kernel, dim3(nblocks(d, 256)), dim3(256), 0, st, F, int(d), eta);
      QC_HIP(hipGetLastError());
    } else {
      const double er = std::exp(m_n.x / double(s)), ph = m_n.y / double(s);
      const double2 eta = make_double2(er * std::cos(ph), er * std::sin(ph));
      QC_HIP(hipMemcpyAsync(X, F, size_t(d) * 16, hipMemcpyDeviceToDevice, st));
      double2* cur = X;
      double2* nxt = Y;
      for (int64_t step = 0; step < s; ++step) {
        for (int j = 1; j <= m; ++j) {
          LaunchTimer tm;
          tm.begin(st);
          const double coef = 1.0 / (double(s) * double(j));
          const int lst = j == m ? 1 : 0;
          if (mode == 0) {
            hipLaunchKernelGGL(action_term_kernel<C2>, dim3(nblocks(d, 4)), dim3(256), 0, st, Om + n * dd, int(d),
                               cur, nxt, F, coef, m_n, lst, eta);
          } else {
            const unsigned tiles = unsigned(nb) * unsigned(nb + 1) / 2;
            hipLaunchKernelGGL(action_tile_kernel<C2>, dim3(tiles), dim3(256), 0, st, Om + n * dd, int(d), nb, cur,
                               P);
            hipLaunchKernelGGL(action_finish_kernel, dim3(4 * unsigned(nb)), dim3(256), 0, st, int(d), nb, cur, nxt,
                               F, P, coef, m_n, lst, eta);
          }
          // one complex multiply-add per matrix element; the whole matrix, or
          // its upper triangle with the diagonal, is read once
          const double elems = mode == 0 ? double(dd) : 0.5 * double(d) * double(d + 1);
          tm.end(st, KERNEL_ACTION, 8.0 * double(dd), elems * sizeof(C2) + 4.0 * 16.0 * double(d));
          std::swap(cur, nxt);
        }
      }
      QC_HIP(hipGetLastError());
    }
    if (t) QC_HIP(hipMemcpyAsync(t + (n + 1) * d, F, size_t(d) * 16, hipMemcpyDeviceToDevice, st));
  }
  return QCHEFF_OK;
}

// y = U x: a workgroup per row with 16-byte row loads where the rows are
// 16-byte aligned (complex128, or complex64 with an even d), about eight loads
// per thread (64 to 512 threads per row); one element per lane per step
// otherwise.
template <typename C2>
void launch_matvec(const C2* U, const double2* x, double2* y, int64_t d, hipStream_t st) {
  if ((sizeof(C2) == 16 || d % 2 == 0) && reinterpret_cast<uintptr_t>(U) % 16 == 0) {
    const int64_t pieces = sizeof(C2) == 16 ? d : d / 2;
    const dim3 grid{unsigned(d)};
    if (pieces <= 512)
      hipLaunchKernelGGL((matvec_rows_kernel<C2, 64>), grid, dim3(64), 0, st, U, x, y, int(d));
    else if (pieces <= 1024)
      hipLaunchKernelGGL((matvec_rows_kernel<C2, 128>), grid, dim3(128), 0, st, U, x, y, int(d));
    else if (pieces <= 2048)
      hipLaunchKernelGGL((matvec_rows_kernel<C2, 256>), grid, dim3(256), 0, st, U, x, y, int(d));
    else
      hipLaunchKernelGGL((matvec_rows_kernel<C2, 512>), grid, dim3(512), 0, st, U, x, y, int(d));
  } else {
    hipLaunchKernelGGL(matvec_kernel<C2>, dim3(nblocks(d, 4)), dim3(256), 0, st, U, x, y, int(d));
  }
}

template <typename T>
int run_propagate(const void* Uv, int64_t M, int64_t d, int mode, void* x, void* traj, void* ws, hipStream_t st) {
  using C2 = typename Cx<T>::t;
  const C2* U = static_cast<const C2*>(Uv);
  const int64_t dd = d * d;
  if (mode == QCHEFF_STATE) {
    double2* psi = static_cast<double2*>(x);
    double2* t = static_cast<double2*>(traj);
    double2* buf[2] = {static_cast<double2*>(ws), static_cast<double2*>(ws) + d};
    if (t) QC_HIP(hipMemcpyAsync(t, psi, size_t(d) * 16, hipMemcpyDeviceToDevice, st));
    const double2* cur = psi;
    for (int64_t n = 0; n < M; ++n) {
      double2* nxt = t ? t + (n + 1) * d : buf[n & 1];
      launch_matvec<C2>(U + n * dd, cur, nxt, d, st);
      QC_HIP(hipGetLastError());
      cur = nxt;
    }
    if (M > 0) QC_HIP(hipMemcpyAsync(psi, cur, size_t(d) * 16, hipMemcpyDeviceToDevice, st));
    return QCHEFF_OK;
  }
  // PRODUCT: binary tree, out[i] = in[2i+1] in[2i]; an odd last matrix is carried.
  C2* P = static_cast<C2*>(x);
  if (M == 0) {
    // identity: a K = 0 product with gamma = 1 writes every element
    auto p = gemm_params<T>(int(d), int(d), 0, 1);
    p.C = P; p.ldc = d; p.sC = 0; p.alpha = T(0); p.gamma = T(1);
    p.A = P; p.B = P; p.lda = d; p.ldb = d;
    QC_HIP((launch_cgemm<T>(p, st)));
    return QCHEFF_OK;
  }
  const size_t mat = align256(size_t(dd) * sizeof(C2));
  C2* bufs[2] = {static_cast<C2*>(ws), reinterpret_cast<C2*>(static_cast<char*>(ws) + size_t((M + 1) / 2) * mat)};
  const int64_t ldm = int64_t(mat / sizeof(C2));  // matrix stride inside the tree buffers
  const C2* in = U;
  int64_t in_stride = dd, cnt = M;
  int which = 0;
  while (cnt > 1) {
    C2* out = bufs[which];
    const int64_t pairs = cnt / 2;
    auto p = gemm_params<T>(int(d), int(d), int(d), int(pairs));
    p.A = in + in_stride; p.lda = d; p.sA = 2 * in_stride;
    p.B = in; p.ldb = d; p.sB = 2 * in_stride;
    p.C = out; p.ldc = d; p.sC = ldm;
    QC_HIP((launch_cgemm<T>(p, st)));
    if (cnt & 1)
      QC_HIP(hipMemcpyAsync(out + pairs * ldm, in + (cnt - 1) * in_stride, size_t(dd) * sizeof(C2),
                            hipMemcpyDeviceToDevice, st));
    in = out;
    in_stride = ldm;
    cnt = pairs + (cnt & 1);
    which ^= 1;
  }
  QC_HIP(hipMemcpyAsync(P, in, size_t(dd) * sizeof(C2), hipMemcpyDeviceToDevice, st));
  return QCHEFF_OK;
}

}  // namespace
}  // namespace qcheff

using namespace qcheff;

extern "C" {

int qcheff_magnus_coeffs(const double* u, int64_t K, int64_t N, double dt_sample, int64_t M, int order, double* c1,
                         double* c2, void* stream) {
  Check c = check_coeffs(u, K, N, dt_sample, M, order, c1, c2);
  if (c.status) return fail(c);
  return run_coeffs(u, K, N, dt_sample, M, order, c1, c2, static_cast<hipStream_t>(stream));
}

int qcheff_magnus_generators(const void* H0, const void* Hk, int64_t d, int64_t K, int op_dtype, const double* c1,
                             const double* c2, int64_t M, double dt_interval, int order, int out_dtype, void* omega,
                             void* ws, size_t ws_bytes, unsigned flags, void* stream) {
  Check c = check_generators(H0, Hk, d, K, op_dtype, c1, c2, M, dt_interval, order, out_dtype, omega, ws, ws_bytes,
                             flags);
  if (c.status) return fail(c);
  return run_generators(static_cast<const double2*>(H0), static_cast<const double2*>(Hk), d, K, c1, c2, M,
                        dt_interval, order, out_dtype, omega, ws, flags, static_cast<hipStream_t>(stream));
}

int qcheff_expm_batched(const void* omega, int64_t batch, int64_t d, int dtype, void* U, int32_t* s_out, void* ws,
                        size_t ws_bytes, void* stream) {
  const bool skew = (dtype & QCHEFF_SKEW_HERMITIAN) != 0;
  const bool refine = (dtype & QCHEFF_UNITARY_REFINE) != 0;
  const bool out64 = (dtype & QCHEFF_OUT_C128) != 0;
  const int bound = ((dtype >> 16) & 0xff) - 1;   // -1: none
  dtype &= ~(QCHEFF_SKEW_HERMITIAN | QCHEFF_UNITARY_REFINE | QCHEFF_OUT_C128 | (0xff << 16));
  const bool bf16x3 = dtype == QCHEFF_C64_BF16X3;
  if (bf16x3) dtype = QCHEFF_C64;
  if (refine && (dtype != QCHEFF_C64 || !skew))
    return fail(QCHEFF_EINVAL, "QCHEFF_UNITARY_REFINE takes QCHEFF_C64 (or _BF16X3) with QCHEFF_SKEW_HERMITIAN");
  if (out64 && !refine) return fail(QCHEFF_EINVAL, "QCHEFF_OUT_C128 needs QCHEFF_UNITARY_REFINE");
  Check c = check_expm(omega, batch, d, dtype, U, ws, ws_bytes, out64 ? QCHEFF_C128 : dtype);
  if (c.status) return fail(c);
  if (batch == 0) return QCHEFF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (bound < 0 && d > kSmallD) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    QC_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(Check::fail(QCHEFF_EUNSUPPORTED,
                              "qcheff_expm_batched: a stream under graph capture needs QCHEFF_SQUARING_BOUND(n)"));
  }
  return dtype == QCHEFF_C128
             ? run_expm<double>(omega, batch, d, U, s_out, ws, ws_bytes, dtype, skew, bound, false, false, false, st)
             : run_expm<float>(omega, batch, d, U, s_out, ws, ws_bytes, dtype, skew, bound, bf16x3, refine, out64,
                               st);
}

int qcheff_expm_grouped(int G, const void* const* omega, const int64_t* batch, const int64_t* d, int dtype,
                        void* const* U, int32_t* const* s_out, void* ws, size_t ws_bytes, void* stream) {
  const bool skew = (dtype & QCHEFF_SKEW_HERMITIAN) != 0;
  const bool refine = (dtype & QCHEFF_UNITARY_REFINE) != 0;
  const bool out64 = (dtype & QCHEFF_OUT_C128) != 0;
  const int bound = ((dtype >> 16) & 0xff) - 1;   // -1: none
  dtype &= ~(QCHEFF_SKEW_HERMITIAN | QCHEFF_UNITARY_REFINE | QCHEFF_OUT_C128 | (0xff << 16));
  const bool bf16x3 = dtype == QCHEFF_C64_BF16X3;
  if (bf16x3) dtype = QCHEFF_C64;
  if (refine && (dtype != QCHEFF_C64 || !skew))
    return fail(QCHEFF_EINVAL, "QCHEFF_UNITARY_REFINE takes QCHEFF_C64 (or _BF16X3) with QCHEFF_SKEW_HERMITIAN");
  if (out64 && !refine) return fail(QCHEFF_EINVAL, "QCHEFF_OUT_C128 needs QCHEFF_UNITARY_REFINE");
  Check c = check_expm_grouped(G, omega, batch, d, dtype, U, ws, ws_bytes, out64 ? QCHEFF_C128 : dtype);
  if (c.status) return fail(c);
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool any_big = false;
  for (int g = 0; g < G; ++g) any_big = any_big || (batch[g] > 0 && d[g] > kSmallD);
  if (bound < 0 && any_big) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    QC_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(Check::fail(QCHEFF_EUNSUPPORTED,
                              "qcheff_expm_grouped: a stream under graph capture needs QCHEFF_SQUARING_BOUND(n)"));
  }
  return dtype == QCHEFF_C128
             ? run_expm_grouped<double>(G, omega, batch, d, U, s_out, ws, ws_bytes, dtype, skew, bound, false, false,
                                        false, st)
             : run_expm_grouped<float>(G, omega, batch, d, U, s_out, ws, ws_bytes, dtype, skew, bound, bf16x3, refine,
                                       out64, st);
}

int qcheff_propagate(const void* U, int64_t M, int64_t d, int dtype, int mode, void* x, void* traj, void* ws,
                     size_t ws_bytes, void* stream) {
  Check c = check_propagate(U, M, d, dtype, mode, x, traj, ws, ws_bytes);
  if (c.status) return fail(c);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == QCHEFF_C128 ? run_propagate<double>(U, M, d, mode, x, traj, ws, st)
                              : run_propagate<float>(U, M, d, mode, x, traj, ws, st);
}

int qcheff_propagate_state_noalloc(const void* U, int64_t M, int64_t d, int dtype, void* x, void* traj,
                                   void* stream) {
  Check c = check_propagate(U, M, d, dtype, QCHEFF_STATE, x, traj, nullptr, 0, /*ws_given=*/false);
  if (c.status) return fail(c);
  if (2 * d > kScratchVecs)
    return fail(QCHEFF_EINVAL, "qcheff_propagate_state_noalloc: d exceeds the 16384 its scratch holds");
  double2* ws = nullptr;
  if (int r = scratch_for_current_device(&ws)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == QCHEFF_C128 ? run_propagate<double>(U, M, d, QCHEFF_STATE, x, traj, ws, st)
                              : run_propagate<float>(U, M, d, QCHEFF_STATE, x, traj, ws, st);
}

int qcheff_propagate_action(const void* omega, int64_t M, int64_t d, int dtype, void* x, void* traj, double tol,
                            void* ws, size_t ws_bytes, void* stream) {
  const bool skew = (dtype & QCHEFF_SKEW_HERMITIAN) != 0;
  dtype &= ~QCHEFF_SKEW_HERMITIAN;
  Check c = check_action(omega, M, d, dtype, x, tol, ws, ws_bytes);
  if (c.status) return fail(c);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == QCHEFF_C128 ? run_action<double>(omega, M, d, x, traj, tol, ws, ws_bytes, skew, st)
                              : run_action<float>(omega, M, d, x, traj, tol, ws, ws_bytes, skew, st);
}

int qcheff_npad_eliminate(void* H, int64_t d, int dtype, const int64_t* pairs, int64_t P, void* ws, size_t ws_bytes,
                          void* stream) {
  Check c = check_npad(H, d, dtype, P, pairs, ws, ws_bytes);
  if (c.status) return fail(c);
  NpadWs w;
  if (!carve_npad(ws, ws_bytes, P, d, w)) return fail(QCHEFF_EWORKSPACE, "workspace carving failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == QCHEFF_C128 ? run_npad_eliminate(static_cast<double2*>(H), d, pairs, P, w, st)
                              : run_npad_eliminate(static_cast<float2*>(H), d, pairs, P, w, st);
}

int qcheff_npad_largest(const void* H, int64_t d, int dtype, int64_t* ij_out, double* mag_out, void* ws,
                        size_t ws_bytes, void* stream) {
  Check c = check_npad(H, d, dtype, 0, ij_out, ws, ws_bytes);
  if (c.status) return fail(c);
  if (!ij_out) return fail(QCHEFF_EINVAL, "ij_out must not be NULL");
  NpadWs w;
  if (!carve_npad(ws, ws_bytes, 0, d, w)) return fail(QCHEFF_EWORKSPACE, "workspace carving failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == QCHEFF_C128 ? run_npad_largest(static_cast<const double2*>(H), d, ij_out, mag_out, w, st)
                              : run_npad_largest(static_cast<const float2*>(H), d, ij_out, mag_out, w, st);
}

int qcheff_propagate_batched(const void* U, int64_t B, int64_t M, int64_t d, int dtype, void* x, void* stream) {
  Check c = check_propagate_batched(U, B, M, d, dtype, x);
  if (c.status) return fail(c);
  if (B == 0 || M == 0) return QCHEFF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t lds = size_t(2 * d) * sizeof(double2);
  if (dtype == QCHEFF_C128)
    hipLaunchKernelGGL(chain_batched_kernel<double2>, dim3(unsigned(B)), dim3(256), lds, st,
                       static_cast<const double2*>(U), static_cast<double2*>(x), int(M), int(d));
  else
    hipLaunchKernelGGL(chain_batched_kernel<float2>, dim3(unsigned(B)), dim3(256), lds, st,
                       static_cast<const float2*>(U), static_cast<double2*>(x), int(M), int(d));
  QC_HIP(hipGetLastError());
  return QCHEFF_OK;
}

size_t qcheff_workspace_bytes(int fn, int64_t batch, int64_t d, int64_t K, int order, int dtype) {
  return workspace_bytes(fn, batch, d, K, order, dtype);
}

const char* qcheff_last_error(void) { return g_last_error.c_str(); }

int qcheff_sync_status(void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  QC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(QCHEFF_EDEVICE, "device index out of range");
  unsigned w = 0;
  {
    // take and clear the word on the stream (after its earlier work), then read it
    std::lock_guard<std::mutex> lk(g_status_mu);
    hipLaunchKernelGGL(take_status_kernel, dim3(1), dim3(1), 0, st);
    QC_HIP(hipGetLastError());
    QC_HIP(hipMemcpyFromSymbolAsync(&w, HIP_SYMBOL(status_taken), sizeof(w), 0, hipMemcpyDeviceToHost, st));
    QC_HIP(hipStreamSynchronize(st));
  }
  w |= g_host_status[dev].exchange(0);
  if (w & STATUS_NONFINITE) return fail(QCHEFF_ENONFINITE, "a generator or its norm was not finite");
  if (w & STATUS_ZERO_PIVOT) return fail(QCHEFF_ENONFINITE, "a Pade denominator had a zero pivot");
  if (w & STATUS_BAD_PAIRS)
    return fail(QCHEFF_EINVAL, "qcheff_npad_eliminate: pairs overlapped or left [0, d) and were left alone");
  return QCHEFF_OK;
}

int qcheff_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (auto& t : g_timed) give_events_locked(t);
  g_timed.clear();
  g_timing.store(on ? 1 : 0);
  return QCHEFF_OK;
}

int qcheff_timing_read(int kernel, int64_t* launches, double* total_ms, double* flops, double* bytes) {
  if (!launches || !total_ms || !flops || !bytes) return fail(QCHEFF_EINVAL, "NULL output pointer");
  std::lock_guard<std::mutex> lk(g_timing_mu);
  int64_t n = 0;
  double ms = 0.0, fl = 0.0, by = 0.0;
  std::vector<TimedLaunch> keep;
  for (auto& t : g_timed) {
    if (t.kernel != kernel) {
      keep.push_back(t);
      continue;
    }
    float e = 0.f;
    if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&e, t.a, t.b) != hipSuccess)
      return fail(QCHEFF_EDEVICE, "reading a timing event failed");
    ms += e;
    fl += t.flops;
    by += t.bytes;
    ++n;
    give_events_locked(t);
  }
  g_timed.swap(keep);
  *launches = n;
  *total_ms = ms;
  *flops = fl;
  *bytes = by;
  return QCHEFF_OK;
}

}  // extern "C"
