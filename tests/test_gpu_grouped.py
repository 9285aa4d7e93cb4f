"""qcheff_expm_grouped: several batches of different dimension in one call,
every product stage one launch over all groups.  Checked against
the oracle (exp by eigendecomposition, oracle/magnus.py) per item, against
qcheff_expm_batched per group, and for its own invariants: the result does not
depend on how the workspace cuts the groups into rounds, a non-finite item
touches no other, and the squaring bound behaves as in qcheff_expm_batched.

Tolerances are those of the expm parity tests (tests/test_gpu_parity.py):
per-item infidelity 1e-12 (FP64) or 1e-6 (FP32 products, refined), unrefined
FP32 max(1e-6, 4 2^s u32); against qcheff_expm_batched bit for bit (every
tile shape accumulates each element in the same order)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl
from tests.test_gpu_parity import DEV, expm_mode, gpu, host, inf_tol, say

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2411_09982_amd")

# (d, batch); d = 20 runs in the fused one-workgroup kernel, d = 130 has a ragged tile
GROUPS = [(20, 5), (40, 7), (64, 6), (100, 4), (130, 3)]


def _inputs(dtype, seed=0):
    oms, refs, seens = [], [], []
    for k, (d, B) in enumerate(GROUPS):
        norms = np.geomspace(0.05, 300.0, B)
        Om = wl.random_skew_hermitian_batch(B, d, norms, config_id=900 + 10 * seed + k)
        refs.append(oracle.expm_skew_hermitian(Om))
        seens.append(Om.astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else Om)
        oms.append(gpu(Om).to(dtype))
    return oms, refs, seens


@pytest.mark.parametrize("mode", ["general", "skew", "refined_c128"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_grouped_matches_oracle_and_batched(dtype, mode):
    kw = expm_mode(mode, dtype)
    if kw is None:
        pytest.skip("the FP64 path takes no refinement")
    say(f"expm grouped {dtype} {mode}: groups {GROUPS}")
    q.sync_status()
    oms, refs, seens = _inputs(dtype)
    Us, ss = q.expm_grouped([o.clone() for o in oms], **kw)
    torch.cuda.synchronize()
    refined = kw["unitary_refine"]
    for (d, B), U, s, ref, seen, om in zip(GROUPS, Us, ss, refs, seens, oms):
        s_ref = [oracle.scaling_exponent(x, shift=(dtype == torch.complex128)) for x in seen]
        assert list(host(s)) == s_ref, d
        Ug = host(U).astype(np.complex128)
        inf = np.abs(oracle.propagator_infidelity(ref, Ug))
        tol = inf_tol(dtype, np.array(s_ref), refined=refined)
        say(f"  d={d}: max infidelity {inf.max():.2e}")
        assert np.all(inf <= tol), (d, inf)
        if dtype == torch.complex128:
            assert np.abs(Ug - ref).max() <= 1e-10
        # the same group alone through qcheff_expm_batched, whose products may take
        # another tile: every tile shape accumulates in the same order, so the bits agree
        U1, s1 = q.expm_batched(om.clone(), **kw)
        torch.cuda.synchronize()
        assert torch.equal(s1, s) and torch.equal(U1, U), d
    assert q.sync_status() == q.OK


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_grouped_rounds_do_not_change_results(dtype):
    # a workspace of one item per group runs as many rounds as the largest batch;
    # one that holds everything runs one: the bits agree
    say(f"expm grouped rounds {dtype}")
    oms, _, _ = _inputs(dtype, seed=1)
    kw = dict(skew_hermitian=True, unitary_refine=dtype == torch.complex64, out_c128=dtype == torch.complex64)
    code = q.C64 if dtype == torch.complex64 else q.C128
    one = sum(q.workspace_bytes(q.FN_EXPM, 1, d, 1, 1, code) for d, _ in GROUPS if d > 32)
    ws = torch.empty(one, dtype=torch.uint8, device=DEV)
    Ua, sa = q.expm_grouped([o.clone() for o in oms], ws=ws, **kw)
    Ub, sb = q.expm_grouped([o.clone() for o in oms], **kw)
    torch.cuda.synchronize()
    for a, b, x, y in zip(Ua, Ub, sa, sb):
        assert torch.equal(x, y) and torch.equal(a, b)
    with pytest.raises(q.QcheffError):
        q.expm_grouped([o.clone() for o in oms], ws=ws[: one - 1], **kw)


def test_grouped_nonfinite_item_and_bound():
    dtype = torch.complex64
    say("expm grouped: a NaN item, and the squaring bound")
    q.sync_status()
    oms, _, _ = _inputs(dtype, seed=2)
    kw = dict(skew_hermitian=True, unitary_refine=True, out_c128=True)
    Uc, sc = q.expm_grouped([o.clone() for o in oms], **kw)
    bad = [o.clone() for o in oms]
    bad[3][1, 2, 3] = float("nan")
    Ub, sb = q.expm_grouped(bad, **kw)
    torch.cuda.synchronize()
    assert int(sb[3][1]) == -1 and torch.isnan(Ub[3][1]).all()
    assert q.sync_status() == q.ENONFINITE and q.sync_status() == q.OK
    for g in range(len(GROUPS)):
        keep = [i for i in range(GROUPS[g][1]) if not (g == 3 and i == 1)]
        assert torch.equal(Ub[g][keep], Uc[g][keep]) and torch.equal(sb[g][keep], sc[g][keep])
    # a bound at the largest count: the same bits, enqueued without a host wait
    smax = max(int(s.max()) for s in sc)
    Ud, sd = q.expm_grouped([o.clone() for o in oms], squaring_bound=smax, **kw)
    torch.cuda.synchronize()
    for a, b, x, y in zip(Ud, Uc, sd, sc):
        assert torch.equal(x, y) and torch.equal(a, b)
    # one squaring short: the items that need more come back as -2 and NaN
    # (the fused kernel of d <= 32 never waits on the host and takes every
    # squaring it needs, bound or not)
    Ue, se = q.expm_grouped([o.clone() for o in oms], squaring_bound=smax - 1, **kw)
    torch.cuda.synchronize()
    for g, (d, B) in enumerate(GROUPS):
        if d <= 32:
            assert torch.equal(se[g], sc[g]) and torch.equal(Ue[g], Uc[g])
            continue
        over = host(sc[g]) > smax - 1
        assert np.array_equal(host(se[g]) == -2, over)
        if over.any():
            assert torch.isnan(Ue[g][torch.from_numpy(over).to(DEV)]).all()


_FORCED_TILE_CHILD = r"""
import json, sys
import numpy as np
import torch
import paper_2411_09982_amd as q
import workloads as wl
groups = [(40, 7), (64, 6), (100, 4), (130, 3)]
out = {}
for dtype in (torch.complex64, torch.complex128):
    print("forced tile, grouped expm", dtype, groups, file=sys.stderr, flush=True)
    oms = [torch.from_numpy(wl.random_skew_hermitian_batch(B, d, np.geomspace(0.05, 300.0, B), config_id=950 + k))
           .to("cuda:0").to(dtype) for k, (d, B) in enumerate(groups)]
    kw = dict(skew_hermitian=True, unitary_refine=dtype == torch.complex64, out_c128=dtype == torch.complex64)
    q.expm_grouped([o.clone() for o in oms], **kw)
    torch.cuda.synchronize()
    q.timing_enable(True)
    Us, ss = q.expm_grouped([o.clone() for o in oms], **kw)
    torch.cuda.synchronize()
    rec = {k: q.timing_read(k)["launches"] for k in (q.KERNEL_GEMM_F32, q.KERNEL_GEMM_BF16X3)}
    q.timing_enable(False)
    same = all(torch.equal(q.expm_batched(o.clone(), **kw)[0], U) for o, U in zip(oms, Us))
    torch.cuda.synchronize()
    out[str(dtype)] = dict(f32=rec[q.KERNEL_GEMM_F32], bf16=rec[q.KERNEL_GEMM_BF16X3], same=same,
                           smax=max(int(s.max()) for s in ss), status=q.sync_status())
print(json.dumps(out), flush=True)
"""


@pytest.mark.parametrize("cfg", [0, 1, 4])
def test_grouped_with_each_tuned_tile(tmp_path, cfg):
    # every tile the tuner may pick, forced through the tune file in a fresh
    # process (the table is read once per process): the grouped call launches
    # each FP32 product stage once over all groups, records it as an FP32 GEMM,
    # and gives the per-group bits
    import json
    import os
    import subprocess
    import sys
    from tests.conftest import ROOT
    say(f"expm grouped with tile configuration {cfg} forced")
    tune = tmp_path / "tune.txt"
    tune.write_text("".join(f"{prec} {d} {cfg}\n" for prec in (q.C64, q.C64 + 100, q.C128, q.C128 + 100)
                            for d in (40, 64, 100, 130)))
    env = dict(os.environ, QCHEFF_TUNE_FILE=str(tune), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", _FORCED_TILE_CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-3000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    c64, c128 = out[str(torch.complex64)], out[str(torch.complex128)]
    assert c64["same"] and c128["same"]
    assert c64["status"] == q.OK and c128["status"] == q.OK
    # one round: six Pade stages, the squaring passes, the refinement's correction
    assert c64["bf16"] == 0 and c64["f32"] == 6 + c64["smax"] + 1, c64
    assert c128["f32"] == 0 and c128["bf16"] == 0
