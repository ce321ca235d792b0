"""GPU energy-window density rows and energy-window LNOs (Sec. II.B: the projector over another
energy window than the occupied states) against the oracle, through the C ABI.

* ldc_window_density on sc27 (plain DC) and on DC-LNO builds of dia216 and fcc_slab: every
  element of W (1e-9, the density bar) and g Tr(W S) against the oracle's state count;
* energy-window LNOs end to end on the gapped diamond: the window above mu, ldc_lno from W with
  lambda_th = 0.5 (4 LNOs per atom, as the oracle finds), then a build with those LNOs: density
  rows, mu and E_band against the oracle's build from its own window rows;
* argument and state errors.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import gpu_build, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["sc27", "dia216", "fcc_slab"])
def test_window_rows_match_oracle(name):
    import torch
    s = synth.small(name)
    print(f"[gpu] window rows {name} atoms={s['n_atoms']}", flush=True)
    fixed = int(s["fixed_k"]) if int(s.get("fixed_k", -1)) >= 0 else None
    dprev = oracle.density_build(s)["D"] if s.get("lno") else None
    ref0 = oracle.density_build(s, dprev=dprev, fixed_rank=fixed)
    win = (ref0["mu"] - 0.3, ref0["mu"] + 0.2, 0.02)
    ref = oracle.density_build(s, dprev=dprev, fixed_rank=fixed, mu=ref0["mu"], window=win)
    g = gpu_build(s, dprev=dprev, fixed_rank=fixed, keep_plan=True)
    plan, (_, S, _) = g["plan"], g["dev"]
    W = torch.zeros_like(S)
    tr = plan.window_density(*win, W)
    torch.cuda.synchronize()
    dw = np.abs(W.cpu().numpy() - ref["W"]).max()
    print(f"  max|dW| {dw:.2e} tr_ws {tr:.10f} oracle count {ref['window_count']:.10f}", flush=True)
    assert dw < 1e-9
    assert abs(tr - ref["window_count"]) < 1e-9 * max(1.0, ref["window_count"])
    assert ref["window_count"] > 1.0
    plan.close()


def test_energy_window_lnos_end_to_end():
    import torch
    s = synth.small("dia216")
    print(f"[gpu] energy-window LNOs {s['name']}", flush=True)
    r0 = oracle.density_build(s)
    win = (r0["mu"], 1e6, s["kT"])
    w_ref = oracle.density_build(s, mu=r0["mu"], window=win)["W"]
    sw = dict(s, lambda_th=0.5, k_min=1, k_max=-1, fixed_k=-1)
    ref = oracle.density_build(sw, dprev=w_ref)
    # device: plain-DC solve, window rows, LNOs from them, then the build with those LNOs
    g0 = gpu_build(s, keep_plan=True)
    plan, (H, S, _) = g0["plan"], g0["dev"]
    W = torch.zeros_like(S)
    plan.window_density(*win, W)
    ranks = plan.lno(S, W, lambda_th=0.5, k_min=1, k_max=-1)
    assert np.all(ranks == 4)
    assert np.array_equal(ranks, np.asarray(ref["ranks"]))
    plan.solve(H, S)
    D = torch.zeros_like(S)
    mu, eb, ne = plan.density(s["n_electrons"], s["kT"], D)
    torch.cuda.synchronize()
    dd = np.abs(D.cpu().numpy() - ref["D"]).max()
    print(f"  max|dD| {dd:.2e} mu {mu:.12f} / {ref['mu']:.12f}", flush=True)
    assert dd < 1e-9
    assert abs(eb - ref["e_band"]) < 1e-10 * s["n_atoms"]
    plan.close()


def test_window_errors():
    import torch
    import paper_1809_05637_amd as ldc
    s = synth.small("sc27")
    plan = ldc.Plan.from_system(s, stream=torch.cuda.current_stream())
    S = to_dev(s["S"])
    W = torch.zeros_like(S)
    with pytest.raises(ldc.LdcError) as e:
        plan.window_density(-1.0, 1.0, 0.01, W)
    assert e.value.status == 8  # LDC_ERR_STATE: no solve yet
    plan.lno(S, None)
    plan.solve(to_dev(s["H"]), S)
    with pytest.raises(ldc.LdcError) as e:
        plan.window_density(1.0, -1.0, 0.01, W)
    assert e.value.status == 1  # LDC_ERR_ARG
    with pytest.raises(ldc.LdcError) as e:
        plan.window_density(-1.0, 1.0, 0.0, W)
    assert e.value.status == 1
    plan.close()
