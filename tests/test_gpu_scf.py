"""GPU toy SCF loop (LNOs regenerated every step, Sec. II.C (i)) against the oracle, through the C ABI.

* ldc_mulliken, ldc_potential and ldc_scf_mix each against the oracle's function on the same
  seeded inputs (uniform and ragged blocks);
* whole trajectories (plain DC on sc27; DC-LNO on dia216 with fixed ranks and on fcc_slab with
  the occupation rule): every step's populations, mu, E_band and density rows.

Tolerances: the density rows at the bar of the build parity tests (1e-9); a population sums
about 3.5e3 products of O(1) entries, so rounding differences in D of 1e-13 give 1e-10 at most;
1e-9 is used.  E_band at 1e-10 Ha per atom.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _plan(s):
    import torch
    import paper_1809_05637_amd as ldc
    return ldc.Plan.from_system(s, stream=torch.cuda.current_stream())


@pytest.mark.parametrize("name", ["fcc_slab", "mixed27"])
def test_mulliken_potential_mix_match_oracle(name):
    """fcc_slab: 9 orbitals per atom with surfaces and vacancies; mixed27: ragged blocks of 1 to
    16 orbitals (the kernels walk the pattern block by block)."""
    import torch
    s = synth.small(name)
    print(f"[gpu] scf kernels {s['name']} atoms={s['n_atoms']}", flush=True)
    rng = np.random.default_rng(7)
    dvals = rng.standard_normal(len(s["S"]))
    v = rng.standard_normal(s["n_atoms"]) * 0.3
    plan = _plan(s)
    S, H0, D = to_dev(s["S"]), to_dev(s["H"]), to_dev(dvals)
    q = torch.zeros(s["n_atoms"], dtype=torch.float64, device=S.device)
    plan.mulliken(D, S, q)
    H = torch.empty_like(H0)
    plan.potential(H0, S, to_dev(v), H)
    torch.cuda.synchronize()
    q_ref = oracle.mulliken(s, dvals)
    assert np.abs(q.cpu().numpy() - q_ref).max() < 1e-11 * max(1.0, np.abs(q_ref).max())
    h_ref = oracle.potential(s, s["H"], v)
    assert np.abs(H.cpu().numpy() - h_ref).max() < 1e-14
    # in place (d_H = d_H0)
    H2 = H0.clone()
    plan.potential(H2, S, to_dev(v), H2)
    torch.cuda.synchronize()
    assert np.abs(H2.cpu().numpy() - h_ref).max() < 1e-14
    # mixing
    q_in = rng.standard_normal(s["n_atoms"])
    q_out = rng.standard_normal(s["n_atoms"])
    q0 = rng.standard_normal(s["n_atoms"])
    qi_d = to_dev(q_in)
    v_d = torch.zeros_like(qi_d)
    res = plan.scf_mix(to_dev(q_out), qi_d, to_dev(q0), 0.7, 0.3, v_d)
    torch.cuda.synchronize()
    q_new = q_in + 0.3 * (q_out - q_in)
    assert res == np.abs(q_out - q_in).max()
    assert np.abs(qi_d.cpu().numpy() - q_new).max() < 1e-15
    assert np.abs(v_d.cpu().numpy() - 0.7 * (q_new - q0)).max() < 1e-14
    plan.close()


@pytest.mark.parametrize("name,steps,U,alpha", [("sc27", 5, 0.5, 0.4), ("dia216", 4, 0.3, 0.3),
                                                ("fcc_slab", 3, 0.2, 0.3)])
def test_scf_trajectory_matches_oracle(name, steps, U, alpha):
    import paper_1809_05637_amd.scf as scf
    s = synth.small(name)
    print(f"[gpu] scf {name} atoms={s['n_atoms']} steps={steps} U={U} alpha={alpha}", flush=True)
    lno = bool(s.get("lno", False))
    fixed = int(s["fixed_k"]) if int(s.get("fixed_k", -1)) >= 0 else None
    ref = oracle.scf_loop(s, U, alpha, steps, lno=lno, fixed_rank=fixed)
    plan = _plan(s)
    hist = scf.scf_loop(plan, to_dev(s["H"]), to_dev(s["S"]), s["n_electrons"], s["kT"], U, alpha, steps,
                        lno=lno, lambda_th=s.get("lambda_th", 0.1), k_min=s.get("k_min", 1), k_max=s.get("k_max", -1),
                        fixed_rank=fixed, keep=True)
    plan.close()
    n = s["n_atoms"]
    for k in range(steps):
        g, r = hist[k], ref[k]
        dq = np.abs(g["q_out"] - r["q_out"]).max()
        dd = np.abs(g["D"] - r["D"]).max()
        print(f"  step {k}: residual {g['residual']:.3e} |dq| {dq:.2e} |dD| {dd:.2e} "
              f"|dmu| {abs(g['mu'] - r['mu']):.2e}", flush=True)
        assert np.abs(g["q_in"] - r["q_in"]).max() < 1e-9, k
        assert dq < 1e-9, k
        assert dd < 1e-9, k
        assert abs(g["mu"] - r["mu"]) < 1e-9, k
        assert abs(g["e_band"] - r["e_band"]) < 1e-10 * n, k
        assert abs(g["residual"] - r["residual"]) < 1e-9, k
    # the loop is doing something: populations move and the residual shrinks
    assert hist[0]["residual"] > 1e-4
    assert hist[-1]["residual"] < hist[0]["residual"]


def test_scf_full_size_kernels_and_sum_rule():
    """Full size (the 3920-atom slab, the benchmark's SCF configuration): two SCF steps; the
    device populations and potential against the oracle's functions applied to the device's
    own density rows and populations, and sum_i q_i = g Tr(D S) = N_e."""
    import torch
    import paper_1809_05637_amd.scf as scf
    s = synth.load_config(2)
    print(f"[gpu] scf full size {s['name']} atoms={s['n_atoms']}", flush=True)
    plan = _plan(s)
    H0, S = to_dev(s["H"]), to_dev(s["S"])
    fixed = int(s["fixed_k"]) if int(s.get("fixed_k", -1)) >= 0 else None
    hist = scf.scf_loop(plan, H0, S, s["n_electrons"], s["kT"], 0.2, 0.3, 2, lno=True,
                        lambda_th=s["lambda_th"], k_min=s["k_min"], k_max=s["k_max"], fixed_rank=fixed, keep=True)
    last = hist[-1]
    q_ref = oracle.mulliken(s, last["D"])
    assert np.abs(last["q_out"] - q_ref).max() < 1e-11 * max(1.0, np.abs(q_ref).max())
    assert abs(last["q_out"].sum() - s["n_electrons"]) < 1e-8 * s["n_electrons"]
    assert abs(last["n_e"] - s["n_electrons"]) < 1e-8 * s["n_electrons"]
    # the potential of the next step from the mixed populations
    q0_d = torch.empty(s["n_atoms"], dtype=torch.float64, device=H0.device)
    plan.reference_populations(s["n_electrons"], q0_d)
    torch.cuda.synchronize()
    q0 = q0_d.cpu().numpy()
    assert np.abs(q0 - oracle.reference_populations(s)).max() <= 1e-14 * s["n_electrons"]
    q_mixed = last["q_in"] + 0.3 * (last["q_out"] - last["q_in"])
    v = 0.2 * (q_mixed - q0)
    H = torch.empty_like(H0)
    plan.potential(H0, S, to_dev(v), H)
    torch.cuda.synchronize()
    assert np.abs(H.cpu().numpy() - oracle.potential(s, s["H"], v)).max() < 1e-14
    plan.close()
    assert hist[1]["residual"] > 0.0
