"""MI355X-native Magnus time-evolution path (arXiv 2411.09982, Sec. 4.1).

Thin Python binding over the C ABI of ``libqcheff_magnus.so`` (include/qcheff.h).
Every step runs in the library's HIP kernels; this module only marshals
arguments: it takes torch tensors on the GPU for device memory, passes their
data pointers and the current HIP stream, and raises ``QcheffError`` on a
non-OK status.  There is no CPU fallback: without the built library every call
raises.

Functions (same names as the C entry points, minus the ``qcheff_`` prefix):
  magnus_coeffs(u, dt_sample, M, order)                 -> c1, c2
  magnus_generators(H0, Hk, c1, c2, dt_interval, order, out_dtype) -> omega
  expm_batched(omega)                                   -> U, s
  expm_grouped([omega_g, ...])                          -> [U_g], [s_g]
  propagate(U, mode, x)                                 -> x (in place)
  sync_status(stream)                                   -> OK or ENONFINITE
and ``evolve(...)``, the four calls in sequence (the paper's evolve()),
``evolve_streamed(...)``, the same with a bounded number of intervals held at a
time, ``evolve_state(...)``, the state-only path through
qcheff_propagate_action, and the NPAD steps of Sec. 3.2 (npad_eliminate,
npad_largest, npad_iterate).
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcheff_magnus.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qcheff.h")

OK, EINVAL, EWORKSPACE, EDEVICE, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
C128, C64, C64_BF16X3 = 1, 2, 3
STATE, PRODUCT = 1, 2
REUSE_BASIS = 1
FN_GENERATORS, FN_EXPM, FN_PROPAGATE, FN_ACTION, FN_NPAD = 1, 2, 3, 4, 5
SKEW_HERMITIAN = 0x100
UNITARY_REFINE = 0x200
OUT_C128 = 0x400
KERNEL_GEMM_F32, KERNEL_GEMM_F64, KERNEL_GEMM_BF16X3, KERNEL_ACTION = 1, 2, 3, 4

_DTYPES = {torch.complex128: C128, torch.complex64: C64}
_TORCH = {C128: torch.complex128, C64: torch.complex64}

_lib = None


class QcheffError(RuntimeError):
    def __init__(self, fn: str, status: int, message: str):
        super().__init__(f"{fn} failed with status {status}: {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2411_09982_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.qcheff_magnus_coeffs.argtypes = [vp, i64, i64, dbl, i64, i32, vp, vp, vp]
    L.qcheff_magnus_generators.argtypes = [vp, vp, i64, i64, i32, vp, vp, i64, dbl, i32, i32, vp, vp,
                                           ctypes.c_size_t, ctypes.c_uint, vp]
    L.qcheff_expm_batched.argtypes = [vp, i64, i64, i32, vp, vp, vp, ctypes.c_size_t, vp]
    L.qcheff_propagate.argtypes = [vp, i64, i64, i32, i32, vp, vp, vp, ctypes.c_size_t, vp]
    L.qcheff_propagate_batched.argtypes = [vp, i64, i64, i64, i32, vp, vp]
    L.qcheff_propagate_state_noalloc.argtypes = [vp, i64, i64, i32, vp, vp, vp]
    L.qcheff_npad_eliminate.argtypes = [vp, i64, i32, vp, i64, vp, ctypes.c_size_t, vp]
    L.qcheff_npad_largest.argtypes = [vp, i64, i32, vp, vp, vp, ctypes.c_size_t, vp]
    L.qcheff_propagate_action.argtypes = [vp, i64, i64, i32, vp, vp, dbl, vp, ctypes.c_size_t, vp]
    L.qcheff_expm_grouped.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
    for f in ("qcheff_magnus_coeffs", "qcheff_magnus_generators", "qcheff_expm_batched", "qcheff_expm_grouped",
              "qcheff_propagate",
              "qcheff_propagate_batched", "qcheff_propagate_action", "qcheff_propagate_state_noalloc",
              "qcheff_npad_eliminate", "qcheff_npad_largest"):
        getattr(L, f).restype = i32
    L.qcheff_workspace_bytes.argtypes = [i32, i64, i64, i64, i32, i32]
    L.qcheff_workspace_bytes.restype = ctypes.c_size_t
    L.qcheff_timing_enable.argtypes = [i32]
    L.qcheff_timing_enable.restype = i32
    L.qcheff_timing_read.argtypes = [i32, vp, vp, vp, vp]
    L.qcheff_timing_read.restype = i32
    L.qcheff_last_error.argtypes = []
    L.qcheff_last_error.restype = ctypes.c_char_p
    L.qcheff_sync_status.argtypes = [vp]
    L.qcheff_sync_status.restype = i32
    _lib = L
    return L


def header_symbols() -> list[str]:
    """Names of the functions include/qcheff.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(qcheff_\w+)\s*\(", text, re.M)))


def _check(fn: str, status: int) -> None:
    if status != OK:
        raise QcheffError(fn, status, lib().qcheff_last_error().decode())


def sync_status(stream=None) -> int:
    """qcheff_sync_status: waits for the stream; OK, ENONFINITE if a generator
    norm was not finite or a Pade denominator had a zero pivot, or EINVAL if NPAD
    pairs overlapped or left the matrix, since the last call (the flags are then
    cleared).  Raises only for a device error."""
    st = lib().qcheff_sync_status(_stream(stream))
    if st not in (OK, ENONFINITE, EINVAL):
        _check("qcheff_sync_status", st)
    return st


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous GPU tensor")
    return t


def workspace_bytes(fn: int, batch: int, d: int, K: int = 1, order: int = 1, dtype: int = C128) -> int:
    return int(lib().qcheff_workspace_bytes(fn, batch, d, K, order, dtype))


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device) if nbytes else None


# --------------------------------------------------------------------- ABI

def c2_columns(K: int, order: int) -> int:
    """Columns of the coefficient table c2: K + K(K-1)/2 second-order ones, and at
    order 3 the (K+1)K(K+3)/2 third-order ones after them."""
    if order < 2:
        return 0
    return K + K * (K - 1) // 2 + ((K + 1) * K * (K + 3) // 2 if order == 3 else 0)


def magnus_coeffs(u: torch.Tensor, dt_sample: float, M: int, order: int, c1=None, c2=None, stream=None):
    """Per-interval coefficients (qcheff_magnus_coeffs).  u: [K][N] float64 on the GPU."""
    _dev(u, "u")
    K, N = u.shape
    if c1 is None:
        c1 = torch.empty((M, K), dtype=torch.float64, device=u.device)
    if order >= 2 and c2 is None:
        c2 = torch.empty((M, c2_columns(K, order)), dtype=torch.float64, device=u.device)
    _check("qcheff_magnus_coeffs", lib().qcheff_magnus_coeffs(
        _ptr(u), K, N, float(dt_sample), M, order, _ptr(c1), _ptr(c2) if order >= 2 else None, _stream(stream)))
    return c1, (c2 if order >= 2 else None)


def magnus_generators(H0, Hk, c1, c2, dt_interval: float, order: int, out_dtype=torch.complex64,
                      omega=None, ws=None, reuse_basis: bool = False, stream=None):
    """Omega_n = -i H-bar_n for every interval (qcheff_magnus_generators).

    Returns (omega, ws); pass ``ws`` back with ``reuse_basis=True`` to skip the
    commutator basis when only the control signals changed.
    """
    _dev(H0, "H0")
    _dev(Hk, "Hk")
    d, K, M = H0.shape[0], Hk.shape[0], c1.shape[0]
    odt = _DTYPES[out_dtype]
    if omega is None:
        omega = torch.empty((M, d, d), dtype=out_dtype, device=H0.device)
    need = workspace_bytes(FN_GENERATORS, 1, d, K, order, C128)
    if ws is None:
        ws = _workspace(need, H0.device)
    _check("qcheff_magnus_generators", lib().qcheff_magnus_generators(
        _ptr(H0), _ptr(Hk), d, K, _DTYPES[H0.dtype], _ptr(c1), _ptr(c2), M, float(dt_interval), order, odt,
        _ptr(omega), _ptr(ws), 0 if ws is None else ws.numel(), REUSE_BASIS if reuse_basis else 0,
        _stream(stream)))
    return omega, ws


def squaring_bound_flag(n: int) -> int:
    """The QCHEFF_SQUARING_BOUND(n) flag bits."""
    if not 0 <= n <= 254:
        raise ValueError("squaring bound must lie in [0, 254]")
    return (n + 1) << 16


def expm_batched(omega, U=None, s_out=None, ws=None, chunk: int | None = None, stream=None,
                 skew_hermitian: bool = False, squaring_bound: int | None = None, bf16x3: bool = False,
                 unitary_refine: bool = False, out_c128: bool = False):
    """U_b = exp(omega_b) by [13/13] Pade scaling and squaring (qcheff_expm_batched).

    ``U`` may be ``omega`` itself.  ``chunk`` caps the items processed at once
    (the workspace is sized for it).  ``skew_hermitian=True`` declares every
    omega_b skew-Hermitian (QCHEFF_SKEW_HERMITIAN): the Hermitian Pade products
    are then formed by halves.  ``squaring_bound=n`` enqueues exactly n squaring
    passes and never waits on the host (graph-capturable); items that need more
    come back with s = -2 and NaN entries.  ``bf16x3=True`` (complex64 only)
    runs the products on the BF16 matrix cores with three-way split operands
    (QCHEFF_C64_BF16X3).  ``unitary_refine=True`` (complex64, skew-Hermitian
    inputs) follows the FP32 squarings with one FP64-Gram Newton step of the
    polar decomposition (QCHEFF_UNITARY_REFINE); with ``out_c128=True`` as well
    the refined U is written in complex128 (QCHEFF_OUT_C128; U then must not
    overlap omega).  Returns (U, s).
    """
    _dev(omega, "omega")
    B, d = omega.shape[0], omega.shape[-1]
    dt = _DTYPES[omega.dtype]
    if bf16x3:
        if dt != C64:
            raise ValueError("bf16x3 products take complex64 matrices")
        dt = C64_BF16X3
    if U is None:
        U = torch.empty(omega.shape, dtype=torch.complex128, device=omega.device) if out_c128 else \
            torch.empty_like(omega)
    if s_out is None:
        s_out = torch.empty(B, dtype=torch.int32, device=omega.device)
    if ws is None:
        ws = _workspace(workspace_bytes(FN_EXPM, max(1, min(B, chunk or B)), d, 1, 1, dt), omega.device)
    _check("qcheff_expm_batched", lib().qcheff_expm_batched(
        _ptr(omega), B, d,
        dt | (SKEW_HERMITIAN if skew_hermitian else 0) | (UNITARY_REFINE if unitary_refine else 0)
        | (OUT_C128 if out_c128 else 0)
        | (0 if squaring_bound is None else squaring_bound_flag(squaring_bound)),
        _ptr(U), _ptr(s_out), _ptr(ws), ws.numel(), _stream(stream)))
    return U, s_out


def expm_grouped_ws_bytes(dims_batches, dtype, chunk: int = 256) -> int:
    """Workspace for qcheff_expm_grouped over (d, batch) groups: the rounds take
    `chunk` items of the group of largest d at a time, and so many of every other
    group (d > 32) that all groups finish in the same number of rounds."""
    code = _DTYPES[dtype] if not isinstance(dtype, int) else dtype
    big = [(d, b) for d, b in dims_batches if d > 32 and b > 0]
    if not big:
        return 0
    dmax, bmax = max(big)
    rounds = -(-bmax // max(1, chunk))
    return sum(workspace_bytes(FN_EXPM, max(1, -(-b // rounds)), d, 1, 1, code) for d, b in big)


def expm_grouped(omegas, Us=None, s_outs=None, ws=None, chunk: int = 256, stream=None,
                 skew_hermitian: bool = False, squaring_bound: int | None = None, bf16x3: bool = False,
                 unitary_refine: bool = False, out_c128: bool = False):
    """exp of several batches of different dimension at once (qcheff_expm_grouped):
    omegas is a list of [B_g][d_g][d_g] tensors of one dtype; the flags are those
    of expm_batched.  Every product stage of a round is one launch over all
    groups.  Returns (Us, ss), lists by group."""
    G = len(omegas)
    if not 1 <= G <= 8:
        raise ValueError("expm_grouped takes 1 to 8 groups")
    for o in omegas:
        _dev(o, "omega")
    dev = omegas[0].device
    dt = _DTYPES[omegas[0].dtype]
    if any(_DTYPES[o.dtype] != dt for o in omegas):
        raise ValueError("every group must have the same dtype")
    if bf16x3:
        if dt != C64:
            raise ValueError("bf16x3 products take complex64 matrices")
        dt = C64_BF16X3
    if Us is None:
        Us = [torch.empty(o.shape, dtype=torch.complex128, device=dev) if out_c128 else torch.empty_like(o)
              for o in omegas]
    if s_outs is None:
        s_outs = [torch.empty(o.shape[0], dtype=torch.int32, device=dev) for o in omegas]
    if ws is None:
        ws = _workspace(max(1, expm_grouped_ws_bytes([(o.shape[-1], o.shape[0]) for o in omegas], dt, chunk)), dev)
    arr = ctypes.c_void_p * G
    i64a = ctypes.c_int64 * G
    om_p = arr(*[_ptr(o) for o in omegas])
    u_p = arr(*[_ptr(u) for u in Us])
    s_p = arr(*[_ptr(x) for x in s_outs])
    batch = i64a(*[o.shape[0] for o in omegas])
    dims = i64a(*[o.shape[-1] for o in omegas])
    _check("qcheff_expm_grouped", lib().qcheff_expm_grouped(
        G, ctypes.cast(om_p, ctypes.c_void_p), ctypes.cast(batch, ctypes.c_void_p), ctypes.cast(dims, ctypes.c_void_p),
        dt | (SKEW_HERMITIAN if skew_hermitian else 0) | (UNITARY_REFINE if unitary_refine else 0)
        | (OUT_C128 if out_c128 else 0)
        | (0 if squaring_bound is None else squaring_bound_flag(squaring_bound)),
        ctypes.cast(u_p, ctypes.c_void_p), ctypes.cast(s_p, ctypes.c_void_p), _ptr(ws),
        0 if ws is None else ws.numel(), _stream(stream)))
    return Us, s_outs


def propagate(U, mode: int, x, traj=None, ws=None, stream=None):
    """Chain the propagators (qcheff_propagate): psi <- U_M ... U_1 psi, or P = U_M ... U_1."""
    _dev(U, "U")
    _dev(x, "x")
    M, d = U.shape[0], U.shape[-1]
    dt = _DTYPES[U.dtype]
    if ws is None:
        ws = _workspace(workspace_bytes(FN_PROPAGATE, M, d, 1, mode, dt), U.device)
    _check("qcheff_propagate", lib().qcheff_propagate(
        _ptr(U), M, d, dt, mode, _ptr(x), _ptr(traj), _ptr(ws), 0 if ws is None else ws.numel(),
        _stream(stream)))
    return x


def propagate_state_noalloc(U, x, traj=None, stream=None):
    """psi <- U_M ... U_1 psi without a workspace (qcheff_propagate_state_noalloc):
    the library's own per-device scratch; calls that overlap on one device race."""
    _dev(U, "U")
    _dev(x, "x")
    M, d = U.shape[0], U.shape[-1]
    _check("qcheff_propagate_state_noalloc", lib().qcheff_propagate_state_noalloc(
        _ptr(U), M, d, _DTYPES[U.dtype], _ptr(x), _ptr(traj), _stream(stream)))
    return x


def propagate_batched(U, x, stream=None):
    """B chains at once (qcheff_propagate_batched): U [B][M][d][d], x [B][d] complex128, in place."""
    _dev(U, "U")
    _dev(x, "x")
    B, M, d = U.shape[0], U.shape[1], U.shape[-1]
    _check("qcheff_propagate_batched", lib().qcheff_propagate_batched(
        _ptr(U), B, M, d, _DTYPES[U.dtype], _ptr(x), _stream(stream)))
    return x


def propagate_action(omega, x, traj=None, tol: float = 0.0, ws=None, stream=None, skew_hermitian: bool = False):
    """psi <- exp(omega[M-1]) ... exp(omega[0]) psi by the truncated Taylor action
    (qcheff_propagate_action); omega [M][d][d] generators, x [d] complex128 in place.
    ``skew_hermitian=True`` declares the generators skew-Hermitian: from d = 2048
    the products then read only their upper triangle (QCHEFF_ACTION_KERNEL=rows|tiles
    overrides the size rule)."""
    _dev(omega, "omega")
    _dev(x, "x")
    M, d = omega.shape[0], omega.shape[-1]
    if ws is None:
        ws = _workspace(workspace_bytes(FN_ACTION, M, d, 1, 1, _DTYPES[omega.dtype]), omega.device)
    _check("qcheff_propagate_action", lib().qcheff_propagate_action(
        _ptr(omega), M, d, _DTYPES[omega.dtype] | (SKEW_HERMITIAN if skew_hermitian else 0), _ptr(x), _ptr(traj),
        float(tol), _ptr(ws), ws.numel(),
        _stream(stream)))
    return x


def evolve_state(H0, Hk, u, dt_sample: float, M: int, order: int, psi0, dtype=torch.complex64,
                 chunk: int = 64, tol: float | None = None, stream=None, hermitian: bool = True):
    """State-only path: coefficients, then per chunk of intervals the generators
    and the Taylor action on the state (no propagator is formed; the generators
    of only `chunk` intervals are held at a time).  Returns psi_M.

    ``tol`` is the truncation tolerance per interval; by default 2^-24 / M for
    complex64 generators (the truncation errors of the whole chain then stay
    below the generators' own rounding, also in the state's norm) and the unit
    roundoff 2^-53 for complex128.  ``hermitian`` states that H0 and every H_k
    are exactly Hermitian, so the generators are exactly skew-Hermitian (the
    products of large d then read half of each)."""
    N = u.shape[1]
    if tol is None:
        tol = 2.0 ** -24 / max(M, 1) if dtype == torch.complex64 else 0.0
    c1, c2 = magnus_coeffs(u, dt_sample, M, order, stream=stream)
    d = H0.shape[0]
    psi = psi0.clone()
    omega = torch.empty((min(chunk, M), d, d), dtype=dtype, device=H0.device)
    gen_ws = None
    act_ws = _workspace(workspace_bytes(FN_ACTION, min(chunk, M), d, 1, 1, _DTYPES[dtype]), H0.device)
    for c0 in range(0, M, chunk):
        c1_ = min(M, c0 + chunk)
        om = omega[: c1_ - c0]
        _, gen_ws = magnus_generators(H0, Hk, c1[c0:c1_], None if c2 is None else c2[c0:c1_],
                                      dt_sample * (N // M), order, dtype, omega=om, ws=gen_ws,
                                      reuse_basis=gen_ws is not None, stream=stream)
        propagate_action(om, psi, tol=tol, ws=act_ws, stream=stream, skew_hermitian=hermitian)
    return psi


def evolve_streamed(H0, Hk, u, dt_sample: float, M: int, order: int, psi0, dtype=torch.complex64,
                    chunk: int = 32, bf16x3: bool = False, hermitian: bool = True, stream=None, progress=None):
    """The propagator path with bounded memory: coefficients once, then per chunk
    of intervals the generators, their exponentials and the state chain (only
    `chunk` generators and propagators are held at a time).  complex64 products
    are refined to unitarity and the propagators kept in complex128.  Returns
    (psi_M, s), s the squaring count of every interval.  ``progress(n)``, if given,
    is called after each chunk has been enqueued with the intervals done so far."""
    N = u.shape[1]
    d = H0.shape[0]
    c1, c2 = magnus_coeffs(u, dt_sample, M, order, stream=stream)
    refine = hermitian and dtype == torch.complex64
    n = min(chunk, M)
    omega = torch.empty((n, d, d), dtype=dtype, device=H0.device)
    U = torch.empty((n, d, d), dtype=torch.complex128, device=H0.device) if refine else omega
    s_all = torch.empty(M, dtype=torch.int32, device=H0.device)
    code = C64_BF16X3 if bf16x3 else _DTYPES[dtype]
    exp_ws = _workspace(workspace_bytes(FN_EXPM, n, d, 1, 1, code), H0.device)
    prop_ws = _workspace(workspace_bytes(FN_PROPAGATE, n, d, 1, STATE, _DTYPES[U.dtype]), H0.device)
    psi = psi0.clone()
    gen_ws = None
    for c0 in range(0, M, chunk):
        c1_ = min(M, c0 + chunk)
        k = c1_ - c0
        _, gen_ws = magnus_generators(H0, Hk, c1[c0:c1_], None if c2 is None else c2[c0:c1_],
                                      dt_sample * (N // M), order, dtype, omega=omega[:k], ws=gen_ws,
                                      reuse_basis=gen_ws is not None, stream=stream)
        expm_batched(omega[:k], U=U[:k], s_out=s_all[c0:c1_], ws=exp_ws, stream=stream,
                     skew_hermitian=hermitian, bf16x3=bf16x3, unitary_refine=refine, out_c128=refine)
        propagate(U[:k], STATE, psi, ws=prop_ws, stream=stream)
        if progress is not None:
            progress(c1_)
    return psi, s_all


# ------------------------------------------------------------------- NPAD

def npad_eliminate(H, pairs, ws=None, stream=None):
    """One NPAD step (qcheff_npad_eliminate): the couplings H[i, j] of the disjoint
    `pairs` ([P][2] int64 on the GPU, or a list of (i, j)) are rotated away in place,
    H <- G H G^dag.  Returns H."""
    _dev(H, "H")
    d = H.shape[0]
    if not isinstance(pairs, torch.Tensor):
        pairs = torch.tensor(list(pairs), dtype=torch.int64).reshape(-1, 2).to(H.device)
    _dev(pairs, "pairs")
    P = pairs.shape[0]
    code = _DTYPES[H.dtype]
    if ws is None:
        ws = _workspace(workspace_bytes(FN_NPAD, P, d, 1, 1, code), H.device)
    _check("qcheff_npad_eliminate", lib().qcheff_npad_eliminate(
        _ptr(H), d, code, _ptr(pairs), P, _ptr(ws), ws.numel(), _stream(stream)))
    return H


def npad_largest(H, ij=None, mag=None, ws=None, stream=None):
    """(i, j), i < j, of the largest |H_ij| as an int64 GPU tensor [1][2] (a `pairs`
    argument for npad_eliminate), and its magnitude (float64 GPU tensor [1])."""
    _dev(H, "H")
    d = H.shape[0]
    code = _DTYPES[H.dtype]
    if ij is None:
        ij = torch.empty((1, 2), dtype=torch.int64, device=H.device)
    if mag is None:
        mag = torch.empty(1, dtype=torch.float64, device=H.device)
    if ws is None:
        ws = _workspace(workspace_bytes(FN_NPAD, 0, d, 1, 1, code), H.device)
    _check("qcheff_npad_largest", lib().qcheff_npad_largest(
        _ptr(H), d, code, _ptr(ij), _ptr(mag), _ptr(ws), ws.numel(), _stream(stream)))
    return ij, mag


def npad_iterate(H, n: int, stream=None):
    """n NPAD steps, each rotating away the largest remaining coupling, all on the
    stream (the pair found by one step feeds the next without a host round trip)."""
    d = H.shape[0]
    ws = _workspace(workspace_bytes(FN_NPAD, 1, d, 1, 1, _DTYPES[H.dtype]), H.device)
    ij = torch.empty((1, 2), dtype=torch.int64, device=H.device)
    mag = torch.empty(1, dtype=torch.float64, device=H.device)
    for _ in range(n):
        npad_largest(H, ij, mag, ws=ws, stream=stream)
        npad_eliminate(H, ij, ws=ws, stream=stream)
    return H


def timing_enable(on: bool) -> None:
    """Start (clearing old records) or stop HIP-event timing of the GEMM kernel launches."""
    _check("qcheff_timing_enable", lib().qcheff_timing_enable(1 if on else 0))


def timing_read(kernel: int) -> dict:
    """Launch count, summed event time (ms), algorithmic flops and bytes of `kernel`'s timed launches."""
    n, ms, fl, by = ctypes.c_int64(0), ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _check("qcheff_timing_read", lib().qcheff_timing_read(kernel, ctypes.byref(n), ctypes.byref(ms),
                                                          ctypes.byref(fl), ctypes.byref(by)))
    return dict(launches=n.value, ms=ms.value, flops=fl.value, bytes=by.value)


def evolve(H0, Hk, u, dt_sample: float, M: int, order: int, psi0=None, dtype=torch.complex64,
           product: bool = False, trajectory: bool = False, chunk: int | None = None, stream=None,
           hermitian: bool = True, bf16x3: bool = False, unitary_refine: bool | None = None,
           out_c128: bool | None = None):
    """The whole path on the GPU: coefficients -> Omega_n -> U_n -> chain.

    Inputs are GPU tensors (H0 [d][d] and Hk [K][d][d] complex128, u [K][N]
    float64, psi0 [d] complex128).  ``hermitian`` states that H0 and every H_k
    are exactly Hermitian (H[c, r] == conj(H[r, c]) bit for bit), as for a
    closed system; the generators are then exactly skew-Hermitian and the
    exponentials use the structured Pade products.  ``bf16x3`` (with
    dtype=complex64) takes the products on the BF16 matrix cores with split
    operands.  ``unitary_refine`` (default: on for complex64 with Hermitian
    operators) refines every FP32 propagator to unitarity after its squarings,
    and ``out_c128`` (default: with the refinement) keeps the refined U in
    complex128.  Returns a dict with c1, c2, U, s and, as asked, psi (final
    state), traj, P.
    """
    N = u.shape[1]
    if unitary_refine is None:
        unitary_refine = hermitian and dtype == torch.complex64
    if out_c128 is None:
        out_c128 = unitary_refine
    c1, c2 = magnus_coeffs(u, dt_sample, M, order, stream=stream)
    omega, _ = magnus_generators(H0, Hk, c1, c2, dt_sample * (N // M), order, dtype, stream=stream)
    U, s = expm_batched(omega, U=None if out_c128 else omega, chunk=chunk, stream=stream, skew_hermitian=hermitian,
                        bf16x3=bf16x3, unitary_refine=unitary_refine, out_c128=out_c128)
    del omega
    out = dict(c1=c1, c2=c2, U=U, s=s)
    if psi0 is not None:
        psi = psi0.clone()
        traj = torch.empty((M + 1, psi.shape[0]), dtype=torch.complex128, device=psi.device) if trajectory else None
        propagate(U, STATE, psi, traj=traj, stream=stream)
        out["psi"] = psi
        if trajectory:
            out["traj"] = traj
    if product:
        P = torch.empty(U.shape[1:], dtype=U.dtype, device=U.device)
        propagate(U, PRODUCT, P, stream=stream)
        out["P"] = P
    return out
