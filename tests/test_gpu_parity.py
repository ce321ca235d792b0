"""GPU path (HIP, through the C ABI) against the CPU oracle on the same seeded inputs.

Bars (FP64 form): max |dD| <= 1e-9, |dE_band| <= 1e-10 Ha/atom, |dmu| <= 1e-9;
spectra per cluster: |d eps| <= 1e-10, |d w| <= 1e-9."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_D = 1e-9
TOL_E = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_05637_amd as ldc
    ldc.load()


def _cmp(s, got, ref, label):
    dD = float(np.abs(got["D"] - ref["D"]).max())
    dE = abs(got["e_band"] - ref["e_band"]) / s["n_atoms"]
    dmu = abs(got["mu"] - ref["mu"])
    print(f"[{label}] max|dD|={dD:.3e} dE/atom={dE:.3e} dmu={dmu:.3e} "
          f"Ne(D)={got['n_e']:.12f} vs {s['n_electrons']}", flush=True)
    assert dD <= TOL_D, dD
    assert dE <= TOL_E, dE
    assert abs(got["n_e"] - s["n_electrons"]) <= 1e-9 * s["n_electrons"]


def test_plain_dc_sc27():
    from gpu_util import gpu_build
    s = synth.small("sc27")
    ref = oracle.density_build(s, workers=1)
    got = gpu_build(s)
    _cmp(s, got, ref, "sc27")


def test_plain_dc_config0():
    from gpu_util import gpu_build
    s = synth.config(0)
    ref = oracle.density_build(s)
    got = gpu_build(s)
    _cmp(s, got, ref, "config0")


def test_cluster_spectra_config0():
    import torch
    from gpu_util import gpu_build
    s = synth.config(0)
    ref = oracle.density_build(s)
    got = gpu_build(s, keep_plan=True)
    plan = got["plan"]
    for i in (0, 13, 63):
        eps, w = plan.cluster_spectrum(i)
        e_ref, w_ref = ref["spectra"][i]
        assert len(eps) == len(e_ref)
        assert np.abs(eps - e_ref).max() <= 1e-10
        assert np.abs(w - w_ref).max() <= 1e-9
    plan.close()


def test_whole_system_equals_exact():
    from gpu_util import gpu_build
    s = synth.small("sc64_whole")
    rho, mu, e = oracle.exact_density(s)
    ex = oracle.exact_density_blocks(s, rho)
    got = gpu_build(s)
    assert np.abs(got["D"] - ex).max() <= TOL_D
    assert abs(got["mu"] - mu) <= 1e-9


@pytest.mark.parametrize("name", ["dia216", "fcc_slab"])
def test_dc_lno(name):
    from gpu_util import gpu_build
    s = synth.small(name)
    r0 = oracle.density_build(s, lno=False)
    ref = oracle.density_build(s, dprev=r0["D"])
    # the GPU's own rank rule must reproduce the oracle's ranks
    got = gpu_build(s, dprev=r0["D"], fixed_rank=(s["fixed_k"] if s["fixed_k"] >= 0 else None))
    assert np.array_equal(got["ranks"], ref["ranks"])
    _cmp(s, got, ref, name + "-lno")
    # plain DC on the same plan inputs
    got0 = gpu_build(s)
    _cmp(s, got0, r0, name + "-plain")


def test_ring_single_orbital():
    """M = 1 per atom, whole-ring clusters: the closed form of the 1D chain."""
    from gpu_util import gpu_build
    s = synth.ring(40, eps=0.1, t=0.8, kT=0.05)
    s["n_electrons"] = 40.0
    ref = oracle.density_build(s, workers=1)
    got = gpu_build(s)
    _cmp(s, got, ref, "ring40")


def test_density_at_fixed_mu():
    from gpu_util import gpu_build
    s = synth.small("sc27")
    ref = oracle.density_build(s, workers=1, mu=0.05, clusters=range(s["n_atoms"]))
    got = gpu_build(s, mu=0.05)
    assert np.abs(got["D"] - ref["D"]).max() <= TOL_D


def test_bracket_error_is_reported():
    import torch
    import paper_1809_05637_amd as ldc
    from gpu_util import to_dev
    s = synth.small("sc27")
    plan = ldc.Plan.from_system(s, stream=torch.cuda.current_stream())
    H, S = to_dev(s["H"]), to_dev(s["S"])
    D = torch.zeros_like(S)
    plan.lno(S, None)
    plan.solve(H, S)
    with pytest.raises(ldc.LdcError) as ei:
        plan.density(10 * s["n_electrons"], s["kT"], D)
    assert ei.value.name == "LDC_ERR_MU_BRACKET"
    # the plan stays usable
    mu, eb, ne = plan.density(s["n_electrons"], s["kT"], D)
    assert abs(ne - s["n_electrons"]) < 1e-9 * s["n_electrons"]
    plan.close()


def test_not_spd_overlap_is_reported_and_plan_recovers():
    """A cluster overlap with a non-positive Cholesky pivot (one atom's onsite S block set to
    -I) is reported as LDC_ERR_NOT_SPD naming a cluster that contains that atom; the same
    plan then builds the intact system to parity."""
    import torch
    import paper_1809_05637_amd as ldc
    from gpu_util import to_dev
    s = synth.small("sc27")
    bad_atom = 5
    S_bad = s["S"].copy()
    rp, col, off, no = s["row_ptr"], s["col"], s["blk_off"], s["n_orb"]
    for b in range(rp[bad_atom], rp[bad_atom + 1]):
        if col[b] == bad_atom:
            m = no[bad_atom]
            S_bad[off[b]: off[b] + m * m] = (-np.eye(m)).ravel()
    plan = ldc.Plan.from_system(s, stream=torch.cuda.current_stream())
    H, Sb, S = to_dev(s["H"]), to_dev(S_bad), to_dev(s["S"])
    D = torch.zeros_like(S)
    plan.lno(Sb, None)
    with pytest.raises(ldc.LdcError) as ei:
        plan.solve(H, Sb)
        plan.density(s["n_electrons"], s["kT"], D)
    assert ei.value.name == "LDC_ERR_NOT_SPD"
    mem_ptr, mem, _ = ldc.regions(s["pos"], s["cell"], s["periodic"], s["n_orb"], s["row_ptr"], s["col"],
                                  s["r_L"], s["kappa"])
    holders = {i for i in range(s["n_atoms"]) if bad_atom in mem[mem_ptr[i]:mem_ptr[i + 1]]}
    assert ei.value.where in holders
    ref = oracle.density_build(s, workers=1)
    plan.lno(S, None)
    plan.solve(H, S)
    mu, eb, ne = plan.density(s["n_electrons"], s["kT"], D)
    torch.cuda.synchronize()
    assert np.abs(D.cpu().numpy() - ref["D"]).max() <= TOL_D
    assert abs(eb - ref["e_band"]) / s["n_atoms"] <= TOL_E
    plan.close()
