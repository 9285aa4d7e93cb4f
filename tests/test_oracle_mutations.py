"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each.

Each mutant is the oracle's own source with one edit (a wrong sign, index,
dropped term or transposed product), loaded as a separate module on the CPU; the
pin tests are then run against it and at least one must fail.
"""
import importlib.util
import inspect
import os
import types

import pytest

import oracle.magnus as om
import tests.test_oracle_pins as pins

MUTANTS = {
    "c20_weight_index": ("w = (s - 1 - 2 * np.arange(s))", "w = (s + 1 - 2 * np.arange(s))"),
    "order2_sign": ("H = H - 0.5j * S", "H = H + 0.5j * S"),
    "chain_transposed": ("P = Un @ P", "P = P @ Un"),
    "exp_sign": ("np.exp(-1j * lam)", "np.exp(1j * lam)"),
    "pair_sign": ("seg[k] * P[l], -(seg[l] * P[k])", "seg[k] * P[l], (seg[l] * P[k])"),
    "drive_index": ("H = H + c1[n, k] * Hk[k]", "H = H + c1[n, k] * Hk[0]"),
    "dropped_sample": ("c1[n, k] = dt * math.fsum(seg[k])", "c1[n, k] = dt * math.fsum(seg[k][1:])"),
    "commutator_swapped": ("comms = [(k, commutator(H0, Hk[k]))", "comms = [(k, commutator(Hk[k], H0))"),
    "missing_conj": ("@ V.conj().T", "@ V.T"),
    "c20_missing_dt": ("c2[n, k] = dt * dt * math.fsum(w * seg[k])", "c2[n, k] = dt * math.fsum(w * seg[k])"),
    "scaling_step": ("        s += 1\n    return s", "        s += 2\n    return s"),
    "state_adjoint": ("psi = Un @ psi", "psi = Un.conj().T @ psi"),
    "drift_dropped": ("H = dt_interval * H0", "H = 0.0 * H0"),
    "infidelity_unnormalised": ("/ (na * nb)", "/ 1.0"),
    "infidelity_no_square": ("abs(np.vdot(a, b)) ** 2", "abs(np.vdot(a, b))"),
    "prop_infidelity_norm_one_side": ("np.abs(tr) ** 2 / (na * nb)", "np.abs(tr) ** 2 / (na * na)"),
    "shift_sign": ("Omega = Omega - mu * np.eye", "Omega = Omega + mu * np.eye"),
    "shift_not_mean": ("complex(np.trace(Omega)) / Omega.shape[-1]", "complex(np.trace(Omega))"),
    "generators_sign": ("return -1j * effective_hamiltonians", "return 1j * effective_hamiltonians"),
    "third_order_sixth": ("out[n] = out[n] - (T[n, a, b, c] / 6.0) * C", "out[n] = out[n] - (T[n, a, b, c] / 3.0) * C"),
    "third_order_sign": ("out[n] = out[n] - (T[n, a, b, c] / 6.0) * C", "out[n] = out[n] + (T[n, a, b, c] / 6.0) * C"),
    "third_order_tie_weight": ("(Q + 0.5 * bc + 0.5 * R + bb / 6.0)", "(Q + bc + 0.5 * R + bb / 6.0)"),
    "third_order_nesting": ("+ commutator(H[c], commutator(H[b], H[a])))", "+ commutator(H[a], commutator(H[b], H[c])))"),
    "state_infidelity_normalised": ("    return 1.0 - abs(np.vdot(a, b)) ** 2\n",
                                    "    return 1.0 - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)\n"),
}


def _load_mutant(name):
    src = inspect.getsource(om)
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, name
    mod = types.ModuleType(f"oracle_mutant_{name}")
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


def _pin_calls():
    for fname, fn in sorted(vars(pins).items()):
        if not fname.startswith("test_") or not callable(fn):
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if params:
            argname, values = params[0].args
            for v in values:
                yield fname, (lambda fn=fn, argname=argname, v=v: fn(**{argname: v}))
        else:
            yield fname, fn


@pytest.mark.filterwarnings("ignore")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, monkeypatch):
    mutant = _load_mutant(name)
    monkeypatch.setattr(pins, "oracle", mutant)
    caught = []
    for fname, call in _pin_calls():
        try:
            call()
        except Exception:
            caught.append(fname)
    assert caught, f"no pin caught mutant {name}"
