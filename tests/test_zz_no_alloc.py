"""The allocation-free density entry point (ldc_density_noalloc) against ldc_density, through
the C ABI: two calls in a row on one GPU, the second on a smaller system, each compared with
ldc_density on the same solve -- the density rows bit for bit and mu, E_band and N_e exactly
(the same kernels in the same order; only the scratch memory differs)."""
import numpy as np
import pytest

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _pair(ldc, s, stream):
    import torch
    H, S = to_dev(s["H"]), to_dev(s["S"])
    plan = ldc.Plan.from_system(s, stream=stream)
    D0 = torch.zeros_like(S)
    plan.lno(S, None)
    plan.solve(H, S)
    plan.density(s["n_electrons"], s["kT"], D0)
    dprev = D0 if s["lno"] else None
    rule = dict(lambda_th=s["lambda_th"], k_min=s["k_min"], k_max=s["k_max"])
    plan.lno(S, dprev, want_ranks=False, **rule)
    plan.solve(H, S)
    Dref = torch.zeros_like(S)
    mu, eb, ne = plan.density(s["n_electrons"], s["kT"], Dref)
    D = torch.full_like(S, 3.0)
    res = torch.full((3,), -1.0, dtype=torch.float64, device=S.device)
    plan.density_noalloc(s["n_electrons"], s["kT"], D, res)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    # the plan's state now holds this call's density: the energy rows follow it
    E = torch.zeros_like(S)
    tr = plan.energy_density(E)
    plan.close()
    return Dref.cpu().numpy(), (mu, eb, ne), D.cpu().numpy(), r, tr


def test_noalloc_matches_density_two_calls(small_systems):
    import torch
    import paper_1809_05637_amd as ldc
    stream = torch.cuda.current_stream()
    for name in ("fcc_slab", "sc27"):  # the second call on a smaller system
        s = small_systems(name)
        print(f"[noalloc] {name}: {s['n_atoms']} atoms", flush=True)
        Dref, (mu, eb, ne), D, r, tr = _pair(ldc, s, stream)
        assert np.array_equal(D, Dref), name
        assert r[0] == mu and r[1] == eb and r[2] == ne, (name, r, mu, eb, ne)
        assert abs(tr - eb) <= 1e-10 * max(1.0, abs(eb))


def test_noalloc_rejects_bad_arguments(small_systems):
    import torch
    import paper_1809_05637_amd as ldc
    s = small_systems("sc27")
    H, S = to_dev(s["H"]), to_dev(s["S"])
    plan = ldc.Plan.from_system(s, stream=torch.cuda.current_stream())
    D = torch.zeros_like(S)
    res = torch.zeros(3, dtype=torch.float64, device=S.device)
    with pytest.raises(ldc.LdcError) as e:
        plan.density_noalloc(s["n_electrons"], s["kT"], D, res)  # before any solve
    assert e.value.name == "LDC_ERR_STATE"
    plan.lno(S, None)
    plan.solve(H, S)
    with pytest.raises(ldc.LdcError) as e:
        plan.density_noalloc(s["n_electrons"], -1.0, D, res)
    assert e.value.name == "LDC_ERR_ARG"
    plan.close()
