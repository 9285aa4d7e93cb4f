/*
 * qcheff.h - C ABI of the MI355X (gfx950) Magnus time-evolution library
 *            libqcheff_magnus.so.
 *
 * The path follows arXiv 2411.09982, Sec. 4.1: a drive Hamiltonian
 *     H(t) = H0 + sum_k u_k(t) H_k                        (Eq. magnus-generic-ham)
 * sampled on N time cells and cut into M equal Magnus intervals.  For interval n
 * the library forms the effective Hamiltonian H-bar_n (first order:
 * Eq. magnus-first-order-term with the coefficients of
 * Eq. magnus-first-order-coeff; second order: the double-commutator term of
 * Eq. magnus-avg), the generator Omega_n = -i H-bar_n, the propagator
 * U_n = exp(Omega_n), and chains the propagators stroboscopically.
 *
 * Conventions shared by every entry point
 *   - hbar = 1.  Times in the caller's unit (ns), frequencies in rad per unit.
 *   - Array pointers are DEVICE pointers unless stated otherwise.  Matrices are
 *     dense, row-major, contiguous; element (i, j) of item b of a [B][d][d]
 *     batch sits at offset (b*d + i)*d + j.  Complex numbers are interleaved
 *     (re, im) pairs: QCHEFF_C128 = two doubles (16 B), QCHEFF_C64 = two floats
 *     (8 B) - the memory layout of std::complex, C99 _Complex and
 *     torch.complex128 / torch.complex64.
 *   - The caller owns every buffer.  The library never allocates or frees caller
 *     memory; scratch memory is the caller's workspace (ws, ws_bytes), sized with
 *     qcheff_workspace_bytes().  It keeps no per-job state between calls.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *     enqueues work on that stream and returns without waiting for it, except
 *     qcheff_expm_batched and qcheff_expm_grouped, which wait once per chunk
 *     (round) for its squaring counts to reach the host (see there).
 *   - Errors: every shape, pointer and workspace check runs on the host before
 *     anything is enqueued; on failure nothing is launched and the call returns
 *     a negative status.  qcheff_last_error() gives a message for the calling
 *     thread's last failure.  A failed launch returns QCHEFF_EDEVICE.
 *   - Calls on distinct streams with distinct buffers may run concurrently.
 */
#ifndef QCHEFF_H
#define QCHEFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define QCHEFF_OK            0
#define QCHEFF_EINVAL       -1  /* bad shape, pointer, order, mode or flag      */
#define QCHEFF_EWORKSPACE   -2  /* workspace missing or too small               */
#define QCHEFF_EDEVICE      -3  /* a HIP call or kernel launch failed           */
#define QCHEFF_ENONFINITE   -4  /* reported by qcheff_sync_status: a non-finite
                                   norm or generator, or a zero pivot, since the
                                   last call of it                              */
#define QCHEFF_EUNSUPPORTED -5  /* valid request the library does not implement */

/* element types */
#define QCHEFF_C128 1           /* complex double; every step in FP64           */
#define QCHEFF_C64  2           /* complex float; products and squarings in FP32
                                   on MFMA, the norm, the scaling choice and the
                                   Pade denominator solve in FP64               */
#define QCHEFF_C64_BF16X3 3     /* qcheff_expm_batched (and its workspace size)
                                   only: complex float storage as QCHEFF_C64,
                                   products and squarings of d > 32 on the BF16
                                   matrix cores with every FP32 operand split in
                                   three BF16 parts (six part products per real
                                   product, FP32 accumulation); norm, scaling
                                   choice and solve in FP64 as for QCHEFF_C64.
                                   d <= 32 runs as QCHEFF_C64.                  */

/* qcheff_expm_batched: OR into dtype to declare every input skew-Hermitian
   (Omega^dag = -Omega, as the Magnus generators are).  The even powers of A and
   the two Pade polynomials are then Hermitian and A W skew-Hermitian, so only the
   upper triangle of each of those products is formed and the lower one is its
   mirror (results exactly (skew-)Hermitian).  Inputs that are not skew-Hermitian
   give wrong results in this mode. */
#define QCHEFF_SKEW_HERMITIAN 0x100

/* qcheff_expm_batched: OR into dtype (QCHEFF_C64 or QCHEFF_C64_BF16X3, together
   with QCHEFF_SKEW_HERMITIAN) to refine every result to unitarity.  The exact
   exponential of a skew-Hermitian matrix is unitary, but each FP32 squaring
   doubles the distance of the computed |eigenvalues| from 1, so after s
   squarings U is off unitarity by about 2^s 2^-24.  With this flag one Newton
   step of the polar decomposition follows the squarings: E = I - U U^dag is
   formed in FP64 from the FP32 values (products on the FP64 matrix cores) and
   U' = U + (1/2) E U (an FP32 product) is written, unitary up to O(|E|^2) and
   the final rounding to complex64.  Costs one FP64 Hermitian product and one
   FP32 product per item.  QCHEFF_EINVAL for QCHEFF_C128 (whose squarings need
   no refinement) or without QCHEFF_SKEW_HERMITIAN. */
#define QCHEFF_UNITARY_REFINE 0x200

/* qcheff_expm_batched: OR into dtype together with QCHEFF_UNITARY_REFINE to
   receive the refined result in FP64: U is then [batch][d][d] complex128 and
   must not overlap omega.  The correction (1/2) E U is added to the FP32 result
   in FP64, so U is unitary up to O(|E|^2) with no final rounding to complex64.
   A chain of M nearly equal propagators (a drift-dominated system) repeats the
   complex64 rounding of each one, and its norm error then grows like M 2^-24;
   complex128 storage removes that term. */
#define QCHEFF_OUT_C128 0x400

/* qcheff_expm_batched: OR QCHEFF_SQUARING_BOUND(n), 0 <= n <= 254, into dtype to
   enqueue exactly n squaring passes without reading the scaling exponents back
   to the host.  The call then never waits on the host and may be captured into
   a HIP graph (without a bound, a stream under capture gets QCHEFF_EUNSUPPORTED
   for d > 32).  An item that needs more than n squarings comes back with
   s_out = -2 and every entry NaN.  d <= 32 never waits; the bound does not
   apply there. */
#define QCHEFF_SQUARING_BOUND(n) ((((n) + 1) & 0xff) << 16)

/* qcheff_propagate modes */
#define QCHEFF_STATE   1
#define QCHEFF_PRODUCT 2

/* qcheff_magnus_generators flags */
#define QCHEFF_REUSE_BASIS 1u

/* qcheff_workspace_bytes selectors */
#define QCHEFF_FN_GENERATORS 1
#define QCHEFF_FN_EXPM       2
#define QCHEFF_FN_PROPAGATE  3
#define QCHEFF_FN_ACTION     4  /* qcheff_propagate_action: batch = M */
#define QCHEFF_FN_NPAD       5  /* qcheff_npad_eliminate / _largest: batch = P */

/*
 * qcheff_magnus_coeffs - per-interval Magnus coefficients of the control
 * signals (Sec. 4.1, Eq. magnus-first-order-coeff; second order from the
 * double integral of Eq. magnus-avg).
 *
 *   u          [K][N] float64, device.  Sample i of control k holds on the cell
 *              [t0 + i*dt_sample, t0 + (i+1)*dt_sample) (zero-order hold).
 *   K, N       controls and samples; K >= 1, N >= 1, N % M == 0.
 *   dt_sample  cell width (> 0, finite).
 *   M          number of intervals; interval n owns samples [n*s, (n+1)*s), s = N/M.
 *   order      1, 2 or 3 (3: K <= 3, else QCHEFF_EUNSUPPORTED).
 *   c1         [M][K] float64, device, written:
 *                c1[n][k] = dt_sample * sum_j u[k][n*s + j].
 *   c2         order 2: [M][K + K(K-1)/2] float64, device, written; ignored
 *              (may be NULL) for order 1.  Columns 0..K-1 weight [H0, H_k]:
 *                c2[n][k] = dt^2 * sum_j (s - 1 - 2j) u_k[j];
 *              column K + p weights [H_k, H_l] for the p-th pair k < l in
 *              row-major order (0,1), (0,2), ..., (1,2), ...:
 *                c2[n][K+p] = dt^2 * sum_j sum_{i<j} (u_k[j] u_l[i] - u_l[j] u_k[i]).
 *              Both are the exact double integrals for a zero-order-hold
 *              signal.  Sums are compensated (Neumaier) in FP64.
 *              Order 3 (the third-order term H-bar^(3) of Eq. magnus-exp): c2 is
 *              [M][P2 + P3], P2 = K + K(K-1)/2 as above and then P3 = (K+1)K(K+3)/2
 *              columns, one per index triple (a, b, c) of {0..K}^3 with a <= c and
 *              not a = b = c, in the order a, then c, then b (index 0 is the drift,
 *              x_0 = 1, and x_k = u_{k-1}):
 *                c3[n][q] = T_abc + T_cba (a < c) or T_aba (a = c),
 *                T_abc = int_{t3<t2<t1 in interval n} x_a(t1) x_b(t2) x_c(t3),
 *              exact for a zero-order-hold signal (cells add dt^3 x_a x_b x_c, ties
 *              half or a sixth of it).
 *   Returns QCHEFF_OK, QCHEFF_EINVAL (shapes, NULL pointers, order, N % M,
 *   dt_sample), QCHEFF_EDEVICE.
 */
int qcheff_magnus_coeffs(const double* u, int64_t K, int64_t N, double dt_sample,
                         int64_t M, int order, double* c1, double* c2, void* stream);

/*
 * qcheff_magnus_generators - Omega_n = -i H-bar_n for M intervals
 * (Eq. magnus-first-order-term; second-order term of Eq. magnus-avg):
 *   H-bar_n = dt_interval H0 + sum_k c1[n][k] H_k
 *             - (i/2) ( sum_k c2[n][k] [H0,H_k] + sum_{k<l} c2[n][K+p(k,l)] [H_k,H_l] )
 *             - (1/6) sum_q c3[n][q] ( [H_a,[H_b,H_c]] + [H_c,[H_b,H_a]] )   (order 3;
 *   q over the triples of qcheff_magnus_coeffs, H_0 the drift).
 *
 *   H0         [d][d] Hermitian, device, op_dtype.
 *   Hk         [K][d][d] Hermitian, device, op_dtype.  Hermiticity is not checked.
 *   op_dtype   QCHEFF_C128 (the library accepts C128 operators only).
 *   c1, c2     as written by qcheff_magnus_coeffs (device); c2 may be NULL for order 1.
 *   M          intervals to form (>= 0).  A caller that streams intervals in
 *              chunks passes c1/c2 offset to the chunk and the chunk's M.
 *   dt_interval  interval length s*dt_sample.
 *   out_dtype  QCHEFF_C128 or QCHEFF_C64 (FP64 assembly, one rounding at the store).
 *   omega      [M][d][d] out_dtype, device, written.
 *   ws         orders 2 and 3: holds the commutator basis, K + K(K-1)/2 matrices
 *              in C128 (order 3: then the P3 nested commutators and two scratch
 *              matrices), computed here (products on MFMA, FP64) unless
 *              flags has QCHEFF_REUSE_BASIS, in which case ws must hold the
 *              basis of an earlier call with the same H0, Hk (the operators are
 *              unchanged when only the control signals change).  Order 1 needs
 *              no workspace.
 *   Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EUNSUPPORTED
 *   (op_dtype other than C128, K > 8, or K > 3 at order 3), QCHEFF_EDEVICE.
 */
int qcheff_magnus_generators(const void* H0, const void* Hk, int64_t d, int64_t K, int op_dtype,
                             const double* c1, const double* c2, int64_t M, double dt_interval,
                             int order, int out_dtype, void* omega, void* ws, size_t ws_bytes,
                             unsigned flags, void* stream);

/*
 * qcheff_expm_batched - U_b = exp(Omega_b) for a batch of d x d matrices by
 * [13/13] Pade scaling and squaring (the exponentiation step of Sec. 4.1; the
 * method is Higham 2005: s_b = smallest s >= 0 with ||Omega_b||_1 / 2^s <= theta13,
 * computed in FP64; A = Omega_b / 2^s; R = q(A)^-1 p(A) by LU with partial
 * pivoting in FP64; U_b = R^(2^s)).  theta13 = 5.371920351148152 is the largest
 * norm at which the [13/13] approximant's backward error stays below 2^-53; both
 * dtypes use it (in FP32 the rounding of the polynomial evaluation, which grows
 * with the norm, outweighs the squaring a larger theta would save).
 *
 *   omega      [batch][d][d], device, dtype.  Any square matrix; the Magnus
 *              generators are skew-Hermitian (dtype | QCHEFF_SKEW_HERMITIAN
 *              halves the Pade products for them).
 *   U          [batch][d][d], device, dtype, written.  Either the same buffer
 *              as omega (the input is consumed) or one that does not overlap it
 *              (QCHEFF_EINVAL otherwise); it also serves as scratch before the
 *              result is written.
 *   s_out      optional [batch] int32, device: the number of squarings used,
 *              -1 where the norm was not finite (that item's U is NaN).
 *   ws         workspace of at least qcheff_workspace_bytes(QCHEFF_FN_EXPM, 1, d, ..);
 *              items are processed in chunks of as many as the workspace holds.
 *   Per chunk the squaring counts go to pinned host memory right after the
 *   scaling; the call waits for them (not for the stream) before it enqueues the
 *   squarings, by which time they are long there.  Everything else is enqueued.
 *   Every launch goes to `stream` (side streams are used by qcheff_expm_grouped
 *   alone).
 *   Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EDEVICE.
 */
int qcheff_expm_batched(const void* omega, int64_t batch, int64_t d, int dtype, void* U,
                        int32_t* s_out, void* ws, size_t ws_bytes, void* stream);

/*
 * qcheff_expm_grouped - qcheff_expm_batched over several batches of different
 * dimension at once: the uneven parameter sweeps the paper runs by
 * exponentiating all Magnus intervals of a job in parallel (Sec. 4.1, 4.3),
 * taken across jobs of different Hilbert-space dimension.
 *
 *   G          number of groups, 1..8.
 *   omega      host array of G device pointers: group g's [batch[g]][d[g]][d[g]]
 *              generators in dtype (as qcheff_expm_batched's omega).
 *   batch, d   host arrays of G sizes.
 *   dtype      as for qcheff_expm_batched, flags included; every group uses it.
 *   U          host array of G device pointers: group g's results (as
 *              qcheff_expm_batched's U, in complex128 with QCHEFF_OUT_C128).
 *              Groups must not overlap one another.
 *   s_out      NULL, or a host array of G device pointers (each NULL or
 *              [batch[g]] int32), as for qcheff_expm_batched.
 *   ws         one workspace for all groups with d[g] > 32, at least the sum of
 *              qcheff_workspace_bytes(QCHEFF_FN_EXPM, 1, d[g], 1, 1, dtype) over
 *              them (groups with d[g] <= 32 run in the fused one-workgroup
 *              kernel and need none).
 *   The groups with d[g] > 32 advance in rounds: each round takes a slice of
 *   every unfinished group, as large as the workspace allows with the same
 *   number of rounds for all.  In a round every product stage (A^2, A^4, A^6,
 *   the two Pade polynomials, the augmented system, each squaring, the two
 *   products of the unitary refinement) is ONE launch over all
 *   groups' tiles (a work list of (group, item, tile) with each group's d and
 *   each item's squaring count); the elementwise steps and the LU solve run per
 *   group.  Split-BF16 products are launched per group.  Results equal those of
 *   qcheff_expm_batched on each group bit for bit (every tile shape accumulates
 *   in the same order).  The groups' solves run side by side on side streams of
 *   the library's own, forked from `stream` and joined back through events.
 *   Without a squaring bound the call waits once per round for the squaring
 *   counts (as qcheff_expm_batched); with QCHEFF_SQUARING_BOUND(n) it never
 *   waits (graph-capturable).
 *   Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EUNSUPPORTED
 *   (graph capture without a bound), QCHEFF_EDEVICE.
 */
int qcheff_expm_grouped(int G, const void* const* omega, const int64_t* batch, const int64_t* d, int dtype,
                        void* const* U, int32_t* const* s_out, void* ws, size_t ws_bytes, void* stream);

/*
 * qcheff_propagate - stroboscopic chain of the interval propagators (Sec. 4.1:
 * the evolution is exact at multiples of the interval; later intervals act
 * on the left).
 *
 *   U          [M][d][d], device, dtype.
 *   mode       QCHEFF_STATE:   x is psi [d] complex128 (always FP64), in: psi_0,
 *                              out: psi_M = U_M ... U_1 psi_0.  Products accumulate
 *                              in FP64.
 *              QCHEFF_PRODUCT: x is P [d][d] in dtype, out: P = U_M ... U_1
 *                              (binary-tree reduction on MFMA).
 *   traj       optional (STATE only) [M+1][d] complex128: psi_0 ... psi_M.
 *   ws         STATE: 2*d complex128; PRODUCT: (ceil(M/2) + ceil(M/4)) d^2 dtype.
 *   Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EDEVICE.
 */
int qcheff_propagate(const void* U, int64_t M, int64_t d, int dtype, int mode, void* x,
                     void* traj, void* ws, size_t ws_bytes, void* stream);

/*
 * qcheff_propagate_state_noalloc - qcheff_propagate in QCHEFF_STATE mode for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * the same results, with the chain's scratch (two state vectors, 2*d
 * complex128) taken from a 512 KiB array the library holds on each device
 * from its first use until the process ends, instead of a workspace.  It
 * allocates nothing and calls no allocating routine.
 *   U, M, d, dtype, x, traj   as for qcheff_propagate (x is psi [d] complex128).
 *   d          1 .. 16384 (QCHEFF_EINVAL beyond: the scratch holds 2 * 16384).
 * Every call on one device shares that device's scratch, which keeps the last
 * call's contents: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.
 * Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EDEVICE.
 */
int qcheff_propagate_state_noalloc(const void* U, int64_t M, int64_t d, int dtype, void* x, void* traj,
                                   void* stream);

/*
 * qcheff_propagate_batched - B independent state chains of equal dimension
 * (parameter sweeps, batches of jobs): chain b computes
 * x[b] <- U[b][M-1] ... U[b][0] x[b], the stroboscopic evolution of Sec. 4.1.
 *
 *   U          [B][M][d][d], device, dtype.
 *   x          [B][d] complex128 (FP64 states, products accumulate in FP64), in/out.
 *   d          1 .. 2048 (each chain's two state vectors are held in LDS).
 *   One workgroup per chain walks all M intervals; no workspace.
 *   Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EDEVICE.
 */
int qcheff_propagate_batched(const void* U, int64_t B, int64_t M, int64_t d, int dtype, void* x, void* stream);

/*
 * qcheff_propagate_action - the stroboscopic state chain of Sec. 4.1 taken from
 * the generators, psi_M = exp(Omega_M) ... exp(Omega_1) psi_0, without forming
 * any exp(Omega_n): each factor acts on the state through a truncated Taylor
 * series (O(d^2) per matrix-vector product instead of O(d^3) per propagator;
 * pays off when d is large and ||Omega_n|| moderate, e.g. many short intervals).
 *
 *   omega      [M][d][d], device, dtype (QCHEFF_C128 or QCHEFF_C64, optionally
 *              | QCHEFF_SKEW_HERMITIAN): the generators.  Any square matrices;
 *              with QCHEFF_SKEW_HERMITIAN (Omega_ji = -conj(Omega_ij), as
 *              qcheff_magnus_generators writes them for Hermitian H0, H_k) the
 *              products for d >= 2048 read the upper triangle (and the 64 x 64
 *              diagonal tiles) only and take the lower triangle as its mirror,
 *              and one row-norm pass gives both norms; the shift reads the
 *              whole diagonal.  Inputs declared skew-Hermitian that are not
 *              give wrong results.
 *   x          [d] complex128, device, in: psi_0, out: psi_M (FP64 state,
 *              products accumulate in FP64).
 *   traj       optional [M+1][d] complex128: psi_0 ... psi_M.
 *   tol        truncation tolerance per interval relative to |psi| (0: the unit
 *              roundoff of dtype, 2^-53 or 2^-24).
 *   Per interval, mu = tr(Omega)/d is split off (exp(Omega) = e^mu exp(Omega -
 *   mu I)); nu = sqrt(||Omega - mu I||_1 ||Omega - mu I||_inf) bounds the
 *   2-norm; the degree m <= 55 and the number of steps s minimise m s subject to
 *   s * sum_{k>m} (nu/s)^k / k! <= tol.  A non-finite generator makes the state
 *   NaN.  The call waits on `stream` once (to read the M shifts and norms).
 *   ws         qcheff_workspace_bytes(QCHEFF_FN_ACTION, M, d, ..) bytes.
 *   Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EDEVICE,
 *   QCHEFF_EUNSUPPORTED (an interval would need more than 2^24 products).
 */
int qcheff_propagate_action(const void* omega, int64_t M, int64_t d, int dtype, void* x, void* traj,
                            double tol, void* ws, size_t ws_bytes, void* stream);

/*
 * qcheff_npad_eliminate - one step of numerical NPAD (Sec. 3.2): the couplings
 * H[i_p][j_p], p < P, of a dense Hermitian H are eliminated in place by
 * H <- G H G^dag, G the product of the two-level Givens rotations of the pairs
 * (Eq. tls-ham).  The rotation of (i, j) diagonalises H restricted to {i, j}
 * without exchanging its two levels: with delta = (H_ii - H_jj)/2, g = |H_ij|,
 * e = H_ij/g, r = sqrt(delta^2 + g^2), c = sqrt((1 + |delta|/r)/2) and
 * s = sign(delta) g / (2 r c) (delta = 0 counts as positive),
 * G_ii = G_jj = c, G_ij = s e, G_ji = -s conj(e).  Rotations of disjoint pairs
 * commute, so all P are one unitary; their parameters come from H before the step.
 *
 *   H          [d][d] Hermitian, device, QCHEFF_C128 or QCHEFF_C64, in place
 *              (arithmetic in FP64; complex64 entries rounded once at the store).
 *   d          2 .. 131072.
 *   pairs      [P][2] int64, device: (i_p, j_p).  Pairs that overlap another pair
 *              or leave [0, d) (i == j included) are left alone and make the next
 *              qcheff_sync_status return QCHEFF_EINVAL; the others are applied.
 *   P          0 .. d/2.
 *   ws         qcheff_workspace_bytes(QCHEFF_FN_NPAD, P, d, 1, 1, dtype) bytes.
 *   Enqueue-only.  Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EDEVICE.
 */
int qcheff_npad_eliminate(void* H, int64_t d, int dtype, const int64_t* pairs, int64_t P, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * qcheff_npad_largest - the coupling NPAD eliminates next when it goes by size
 * (Sec. 3.2: rotating away the largest off-diagonal terms first): (i, j), i < j,
 * of the largest |H_ij| above the diagonal, the first in row-major order among
 * equal magnitudes; a NaN counts as the largest.
 *   ij_out     [2] int64, device, written (the layout of one `pairs` row, so it can
 *              be passed straight to qcheff_npad_eliminate with P = 1).
 *   mag_out    optional [1] double, device: the magnitude.
 *   ws         qcheff_workspace_bytes(QCHEFF_FN_NPAD, 0, d, 1, 1, dtype) bytes.
 *   Enqueue-only.  Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EWORKSPACE, QCHEFF_EDEVICE.
 */
int qcheff_npad_largest(const void* H, int64_t d, int dtype, int64_t* ij_out, double* mag_out, void* ws,
                        size_t ws_bytes, void* stream);

/*
 * qcheff_workspace_bytes - workspace needed by `fn` (QCHEFF_FN_*):
 *   GENERATORS: (batch, K, order, d) -> commutator basis bytes (0 for order 1);
 *   EXPM:       bytes to process `batch` items at once (per-item size x batch);
 *   PROPAGATE:  `batch` is M, `order` carries the mode (QCHEFF_STATE / _PRODUCT).
 * Returns 0 for an invalid selector or shape.
 */
size_t qcheff_workspace_bytes(int fn, int64_t batch, int64_t d, int64_t K, int order, int dtype);

/* Message for the calling thread's last non-OK status (never NULL). */
const char* qcheff_last_error(void);

/*
 * qcheff_sync_status - reports and clears the conditions the library's kernels
 * (and host-side checks) have flagged on the current device since the previous
 * call: a non-finite norm of a generator (the scaling step of the exponential,
 * Sec. 4.1, or the Taylor action), or a zero pivot in the LU of a Pade
 * denominator.  The affected results are NaN (qcheff_expm_batched also marks
 * them with s_out = -1); this call is the one place to learn about it without
 * inspecting them.  The device's flag word is taken and cleared in one atomic
 * step by a kernel enqueued on `stream` (so after the stream's earlier work),
 * then read back; the call waits for `stream`.  A flag that a kernel on
 * another stream sets meanwhile is kept for the next call.  The flags are per
 * device and shared by every stream and thread of the process, so they cannot
 * say which job raised them.
 * Returns QCHEFF_OK, QCHEFF_ENONFINITE, QCHEFF_EINVAL (a qcheff_npad_eliminate call
 * was given pairs that overlapped or left [0, d); those pairs were left alone) or
 * QCHEFF_EDEVICE.
 */
int qcheff_sync_status(void* stream);

/*
 * Kernel timing (instrumentation for throughput and roofline measurements).
 * While enabled, every launch of the library's complex MFMA GEMM kernel is
 * bracketed by a pair of HIP events recorded on the launch stream, together
 * with the launch's algorithmic flop count (8 M N K per active item: a complex
 * multiply-add is 8 real flops) and byte count (operands read once, result
 * written once).
 *   qcheff_timing_enable(1) clears old records and starts recording;
 *   qcheff_timing_enable(0) clears them and stops.
 *   qcheff_timing_read(kernel, ...) waits for the recorded events of `kernel`
 *   (QCHEFF_KERNEL_GEMM_F32 / _F64 / _BF16X3 / _ACTION), returns the number of launches, the summed
 *   event-to-event time in ms and the summed flops and bytes, and releases
 *   those records.  Returns QCHEFF_OK, QCHEFF_EINVAL, QCHEFF_EDEVICE.
 * Recording costs two event records per GEMM launch; leave it off otherwise.
 */
#define QCHEFF_KERNEL_GEMM_F32 1
#define QCHEFF_KERNEL_GEMM_F64 2
#define QCHEFF_KERNEL_GEMM_BF16X3 3
#define QCHEFF_KERNEL_ACTION 4   /* one Taylor term of qcheff_propagate_action: 8 d^2 flops, d^2 elements read */
int qcheff_timing_enable(int on);
int qcheff_timing_read(int kernel, int64_t* launches, double* total_ms, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* QCHEFF_H */
