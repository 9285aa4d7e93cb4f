"""C-ABI checks that need no GPU: the library loads, exports what the header
declares, rejects bad arguments before launching anything, and sizes its
workspaces as documented."""
import ctypes

import pytest

import paper_2411_09982_amd as q

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(q.LIB_PATH),
                                reason="libqcheff_magnus.so not built")


def test_exports_every_header_symbol():
    names = q.header_symbols()
    assert set(names) == {"qcheff_magnus_coeffs", "qcheff_magnus_generators", "qcheff_expm_batched",
                          "qcheff_propagate", "qcheff_workspace_bytes", "qcheff_last_error",
                          "qcheff_timing_enable", "qcheff_timing_read", "qcheff_propagate_batched",
                          "qcheff_propagate_action", "qcheff_sync_status", "qcheff_propagate_state_noalloc",
                          "qcheff_npad_eliminate", "qcheff_npad_largest", "qcheff_expm_grouped"}
    L = q.lib()
    for n in names:
        assert hasattr(L, n), n


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation


def _err():
    return q.lib().qcheff_last_error().decode()


def test_coeffs_validation():
    L = q.lib()
    assert L.qcheff_magnus_coeffs(FAKE, 1, 10, 0.1, 3, 1, FAKE, None, None) == q.EINVAL
    assert "multiple" in _err()
    assert L.qcheff_magnus_coeffs(FAKE, 1, 10, 0.1, 5, 4, FAKE, FAKE, None) == q.EINVAL
    assert "order" in _err()
    assert L.qcheff_magnus_coeffs(FAKE, 1, 10, 0.1, 5, 2, FAKE, None, None) == q.EINVAL
    assert L.qcheff_magnus_coeffs(None, 1, 10, 0.1, 5, 1, FAKE, None, None) == q.EINVAL
    assert L.qcheff_magnus_coeffs(FAKE, 0, 10, 0.1, 5, 1, FAKE, None, None) == q.EINVAL
    assert L.qcheff_magnus_coeffs(FAKE, 1, 10, -0.1, 5, 1, FAKE, None, None) == q.EINVAL
    assert L.qcheff_magnus_coeffs(FAKE, 1, 10, float("nan"), 5, 1, FAKE, None, None) == q.EINVAL
    assert L.qcheff_magnus_coeffs(FAKE, 1, 10, 0.1, 0, 1, FAKE, None, None) == q.EINVAL


def test_generators_validation():
    L = q.lib()
    g = L.qcheff_magnus_generators
    # order 2 without workspace
    assert g(FAKE, FAKE, 4, 1, q.C128, FAKE, FAKE, 3, 0.1, 2, q.C64, FAKE, None, 0, 0, None) == q.EWORKSPACE
    need = q.workspace_bytes(q.FN_GENERATORS, 1, 4, 1, 2, q.C128)
    assert need == 256  # one 4x4 complex128 commutator, rounded up to 256 B
    assert g(FAKE, FAKE, 4, 1, q.C128, FAKE, FAKE, 3, 0.1, 2, q.C64, FAKE, FAKE, need - 1, 0, None) == q.EWORKSPACE
    assert g(FAKE, FAKE, 4, 1, q.C64, FAKE, FAKE, 3, 0.1, 1, q.C64, FAKE, None, 0, 0, None) == q.EUNSUPPORTED
    assert g(FAKE, FAKE, 4, 9, q.C128, FAKE, FAKE, 3, 0.1, 1, q.C64, FAKE, None, 0, 0, None) == q.EUNSUPPORTED
    assert g(FAKE, FAKE, 4, 1, q.C128, FAKE, FAKE, 3, 0.1, 1, 7, FAKE, None, 0, 0, None) == q.EINVAL
    assert g(FAKE, FAKE, 0, 1, q.C128, FAKE, FAKE, 3, 0.1, 1, q.C64, FAKE, None, 0, 0, None) == q.EINVAL
    assert g(FAKE, FAKE, 4, 1, q.C128, FAKE, FAKE, 3, 0.1, 1, q.C64, FAKE, None, 0, 4, None) == q.EINVAL
    assert g(None, FAKE, 4, 1, q.C128, FAKE, FAKE, 3, 0.1, 1, q.C64, FAKE, None, 0, 0, None) == q.EINVAL
    assert g(FAKE, FAKE, 4, 1, q.C128, FAKE, None, 3, 0.1, 2, q.C64, FAKE, FAKE, need, 0, None) == q.EINVAL


def test_expm_grouped_validation():
    # qcheff_expm_grouped: G in [1, 8], the per-group checks of qcheff_expm_batched,
    # and one workspace holding at least one item of every group with d > 32
    L = q.lib()
    e = L.qcheff_expm_grouped
    arr = ctypes.c_void_p * 3
    i64 = ctypes.c_int64 * 3
    cast = lambda x: ctypes.cast(x, ctypes.c_void_p)
    base = FAKE.value
    om = arr(base, base + (1 << 28), base + (2 << 28))
    us = arr(base + (3 << 28), base + (4 << 28), base + (5 << 28))
    dims, batch = i64(20, 40, 100), i64(3, 2, 5)
    need = q.workspace_bytes(q.FN_EXPM, 1, 40, 1, 1, q.C64) + q.workspace_bytes(q.FN_EXPM, 1, 100, 1, 1, q.C64)
    call = lambda G, o=om, b=batch, d=dims, u=us, ws=FAKE, n=need, dt=q.C64: e(
        G, cast(o), cast(b), cast(d), dt, cast(u), None, ws, n, None)
    assert call(0) == q.EINVAL and call(9) == q.EINVAL
    assert e(3, None, cast(batch), cast(dims), q.C64, cast(us), None, FAKE, need, None) == q.EINVAL
    assert e(3, cast(om), cast(batch), None, q.C64, cast(us), None, FAKE, need, None) == q.EINVAL
    # the d = 20 group runs in the fused kernel and needs no workspace; the others one item each
    assert call(3, n=need - 1) == q.EWORKSPACE
    assert call(3, ws=None, n=0) == q.EWORKSPACE
    # per-group checks, with the group named in the message
    bad = i64(20, 0, 100)
    assert call(3, d=bad) == q.EINVAL and b"group 1" in L.qcheff_last_error()
    over = arr(base + (3 << 28), base + (4 << 28), base + (2 << 28) + 64)   # U of group 2 overlaps its omega
    assert call(3, u=over) == q.EINVAL and b"group 2" in L.qcheff_last_error()
    neg = i64(3, -1, 5)
    assert call(3, b=neg) == q.EINVAL
    # the flags of qcheff_expm_batched
    assert call(3, dt=q.C64 | q.UNITARY_REFINE) == q.EINVAL          # refinement needs the skew flag
    assert call(3, dt=q.C128 | q.SKEW_HERMITIAN | q.UNITARY_REFINE) == q.EINVAL
    assert call(3, dt=q.C64 | q.SKEW_HERMITIAN | q.OUT_C128) == q.EINVAL   # complex128 output needs refinement
    # empty groups launch nothing
    zero = i64(0, 0, 0)
    assert call(3, b=zero, ws=None, n=0) == q.OK


def test_expm_validation_and_workspace():
    L = q.lib()
    e = L.qcheff_expm_batched
    assert e(FAKE, 2, 0, q.C64, FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    assert e(FAKE, 2, 8, 5, FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    assert e(FAKE, 2, 8, q.C64, FAKE, None, None, 0, None) == q.EWORKSPACE
    one = q.workspace_bytes(q.FN_EXPM, 1, 8, 1, 1, q.C64)
    two = q.workspace_bytes(q.FN_EXPM, 2, 8, 1, 1, q.C64)
    assert 0 < one < two
    assert e(FAKE, 2, 8, q.C64, FAKE, None, FAKE, one - 1, None) == q.EWORKSPACE
    assert e(None, 2, 8, q.C64, FAKE, None, FAKE, one, None) == q.EINVAL
    assert e(FAKE, -1, 8, q.C64, FAKE, None, FAKE, one, None) == q.EINVAL
    # U is omega itself or a buffer that does not overlap it
    for off in (8, 2 * 8 * 8 * 8 - 8):
        assert e(FAKE, 2, 8, q.C64, ctypes.c_void_p(FAKE.value + off), None, FAKE, 1 << 30, None) == q.EINVAL
        assert e(ctypes.c_void_p(FAKE.value + off), 2, 8, q.C64, FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    # per item: 6 d^2 working matrices + the 2 d^2 FP64 augmented system + pivots
    d = 1000
    c64 = q.workspace_bytes(q.FN_EXPM, 1, d, 1, 1, q.C64)
    c128 = q.workspace_bytes(q.FN_EXPM, 1, d, 1, 1, q.C128)
    assert c64 >= 6 * d * d * 8 + 2 * d * d * 16 and c64 < 6 * d * d * 8 + 2 * d * d * 16 + 8192
    assert c128 >= 6 * d * d * 16 + 2 * d * d * 16
    assert e(FAKE, 0, 8, q.C64, FAKE, None, None, 0, None) == q.OK   # empty batch is a no-op
    # the split-BF16 products take the complex64 layout and workspace
    assert q.workspace_bytes(q.FN_EXPM, 2, 40, 1, 1, q.C64_BF16X3) == q.workspace_bytes(q.FN_EXPM, 2, 40, 1, 1, q.C64)
    assert e(FAKE, 0, 8, q.C64_BF16X3, FAKE, None, None, 0, None) == q.OK
    assert e(FAKE, 2, 8, q.C64_BF16X3, FAKE, None, None, 0, None) == q.EWORKSPACE
    # the skew-Hermitian flag rides on the dtype; other bits stay invalid
    assert e(FAKE, 0, 8, q.C64 | q.SKEW_HERMITIAN, FAKE, None, None, 0, None) == q.OK
    assert e(FAKE, 2, 8, 5 | q.SKEW_HERMITIAN, FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    assert e(FAKE, 2, 8, q.C64 | 0x200, FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    assert e(FAKE, 2, 8, q.C64 | q.SKEW_HERMITIAN, FAKE, None, None, 0, None) == q.EWORKSPACE
    # the squaring bound rides on bits 16..23
    assert e(FAKE, 0, 8, q.C128 | q.squaring_bound_flag(7), FAKE, None, None, 0, None) == q.OK
    assert e(FAKE, 2, 8, 5 | q.squaring_bound_flag(7), FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    assert e(FAKE, 2, 8, q.C64 | (1 << 24), FAKE, None, FAKE, 1 << 30, None) == q.EINVAL
    assert q.squaring_bound_flag(0) == 1 << 16 and q.squaring_bound_flag(254) == 255 << 16
    with pytest.raises(ValueError):
        q.squaring_bound_flag(255)


def test_propagate_validation():
    L = q.lib()
    p = L.qcheff_propagate
    assert p(FAKE, 3, 4, q.C64, 9, FAKE, None, FAKE, 1 << 20, None) == q.EINVAL
    assert p(FAKE, 3, 4, q.C64, q.PRODUCT, FAKE, FAKE, FAKE, 1 << 20, None) == q.EINVAL
    assert p(FAKE, 3, 4, q.C64, q.STATE, None, None, FAKE, 1 << 20, None) == q.EINVAL
    assert p(FAKE, 3, 4, q.C64, q.STATE, FAKE, None, None, 0, None) == q.EWORKSPACE
    assert q.workspace_bytes(q.FN_PROPAGATE, 3, 4, 1, q.STATE, q.C64) == 256
    # product tree: ceil(M/2) + ceil(M/4) matrices of 256-byte-rounded size
    assert q.workspace_bytes(q.FN_PROPAGATE, 5, 4, 1, q.PRODUCT, q.C64) == (3 + 2) * 256
    assert q.workspace_bytes(9, 5, 4, 1, 1, q.C64) == 0


def test_propagate_action_validation():
    L = q.lib()
    a = L.qcheff_propagate_action
    need = q.workspace_bytes(q.FN_ACTION, 3, 10, 1, 1, q.C64)
    # two term vectors, the shifts, the norms and the tile shares, each on a
    # 256-byte boundary
    assert need == 2 * 256 + 256 + 256 + 1024
    assert q.workspace_bytes(q.FN_ACTION, 1000, 4096, 1, 1, q.C128) == 2 * 65536 + 2 * 16128 + 64 * 64 * 64 * 16
    assert q.workspace_bytes(q.FN_ACTION, 3, 10, 1, 1, 9) == 0
    assert a(FAKE, -1, 10, q.C64, FAKE, None, 0.0, FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 0, q.C64, FAKE, None, 0.0, FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 10, 9, FAKE, None, 0.0, FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 10, q.C64, None, None, 0.0, FAKE, need, None) == q.EINVAL
    assert a(None, 3, 10, q.C64, FAKE, None, 0.0, FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 10, q.C64, FAKE, None, -1e-3, FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 10, q.C64, FAKE, None, float("nan"), FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 10, q.C64, FAKE, None, 1.0, FAKE, need, None) == q.EINVAL
    assert a(FAKE, 3, 10, q.C64, FAKE, None, 0.0, FAKE, need - 1, None) == q.EWORKSPACE
    assert a(FAKE, 3, 10, q.C64, FAKE, None, 0.0, None, 0, None) == q.EWORKSPACE
    # M = 0 without a trajectory enqueues nothing
    need0 = q.workspace_bytes(q.FN_ACTION, 0, 10, 1, 1, q.C64)
    assert a(None, 0, 10, q.C64, FAKE, None, 0.0, FAKE, need0, None) == q.OK


def test_propagate_batched_validation():
    L = q.lib()
    p = L.qcheff_propagate_batched
    assert p(FAKE, 2, 3, 0, q.C64, FAKE, None) == q.EINVAL
    assert p(FAKE, 2, 3, 2049, q.C64, FAKE, None) == q.EINVAL
    assert p(FAKE, 2, 3, 8, 9, FAKE, None) == q.EINVAL
    assert p(FAKE, 2, 3, 8, q.C64, None, None) == q.EINVAL
    assert p(None, 2, 3, 8, q.C64, FAKE, None) == q.EINVAL
    assert p(None, 0, 3, 8, q.C64, None, None) == q.OK


def test_timing_api_without_gpu():
    L = q.lib()
    assert L.qcheff_timing_read(1, None, None, None, None) == q.EINVAL
    n, ms, fl, by = ctypes.c_int64(7), ctypes.c_double(1), ctypes.c_double(1), ctypes.c_double(1)
    assert L.qcheff_timing_enable(0) == q.OK
    assert L.qcheff_timing_read(1, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)) == q.OK
    assert n.value == 0 and ms.value == 0.0


def test_no_cpu_fallback_in_binding(monkeypatch, tmp_path):
    # the binding refuses to run without the HIP library
    monkeypatch.setattr(q, "_lib", None)
    monkeypatch.setattr(q, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        q.lib()


def test_propagate_state_noalloc_validation():
    L = q.lib()
    f = L.qcheff_propagate_state_noalloc
    assert f(FAKE, 2, 20000, q.C64, FAKE, None, None) == q.EINVAL       # d beyond the scratch
    assert f(FAKE, 2, 4, q.C64, None, None, None) == q.EINVAL           # no state
    assert f(None, 2, 4, q.C64, FAKE, None, None) == q.EINVAL           # no propagators
    assert f(FAKE, -1, 4, q.C64, FAKE, None, None) == q.EINVAL
    assert f(FAKE, 2, 4, 9, FAKE, None, None) == q.EINVAL


def test_npad_validation():
    L = q.lib()
    need = q.workspace_bytes(q.FN_NPAD, 3, 10, 1, 1, q.C128)
    assert need == 256 + 256 + 256 + 256
    e = L.qcheff_npad_eliminate
    assert e(FAKE, 1, q.C128, FAKE, 0, FAKE, need, None) == q.EINVAL            # d < 2
    assert e(FAKE, 10, q.C128, FAKE, 6, FAKE, need, None) == q.EINVAL           # P > d / 2
    assert e(FAKE, 10, 7, FAKE, 3, FAKE, need, None) == q.EINVAL                # dtype
    assert e(None, 10, q.C128, FAKE, 3, FAKE, need, None) == q.EINVAL           # H
    assert e(FAKE, 10, q.C128, None, 3, FAKE, need, None) == q.EINVAL           # pairs
    assert e(FAKE, 10, q.C128, FAKE, 3, FAKE, need - 1, None) == q.EWORKSPACE
    lg = L.qcheff_npad_largest
    assert lg(FAKE, 10, q.C64, None, None, FAKE, need, None) == q.EINVAL        # ij_out
    assert lg(FAKE, 10, q.C64, FAKE, None, None, 0, None) == q.EWORKSPACE


def test_order3_validation():
    L = q.lib()
    assert L.qcheff_magnus_coeffs(FAKE, 4, 10, 0.1, 5, 3, FAKE, FAKE, None) == q.EUNSUPPORTED   # K > 3
    assert L.qcheff_magnus_coeffs(FAKE, 2, 10, 0.1, 5, 4, FAKE, FAKE, None) == q.EINVAL        # order 4
    assert L.qcheff_magnus_coeffs(FAKE, 2, 10, 0.1, 5, 3, FAKE, None, None) == q.EINVAL        # no c2
    # basis: K + K(K-1)/2 commutators, (K+1)K(K+3)/2 nested ones, two scratch matrices
    assert q.workspace_bytes(q.FN_GENERATORS, 1, 4, 2, 3, q.C128) == (3 + 15 + 2) * 16 * 16
    assert q.workspace_bytes(q.FN_GENERATORS, 1, 4, 4, 3, q.C128) == 0
    g = L.qcheff_magnus_generators
    assert g(FAKE, FAKE, 4, 4, q.C128, FAKE, FAKE, 3, 0.1, 3, q.C64, FAKE, FAKE, 1 << 20, 0, None) == q.EUNSUPPORTED
    assert q.c2_columns(2, 3) == 3 + 15 and q.c2_columns(3, 2) == 6 and q.c2_columns(1, 1) == 0
