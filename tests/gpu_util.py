"""Helpers for the GPU tests: run one density build through the C ABI."""
import numpy as np


def device():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def gpu_build(s, dprev=None, fixed_rank=None, mu=None, plan=None, keep_plan=False, energy=False):
    """One build (ldc_lno, ldc_solve, ldc_density or ldc_density_at, and with energy=True
    ldc_energy_density).  Returns a dict."""
    import torch
    import paper_1809_05637_amd as ldc
    print(f"[gpu] build {s.get('name')} atoms={s['n_atoms']} lno={dprev is not None}", flush=True)
    H, S = to_dev(s["H"]), to_dev(s["S"])
    D = torch.zeros_like(S)
    own = plan is None
    if own:
        plan = ldc.Plan.from_system(s, stream=torch.cuda.current_stream())
    dp = to_dev(dprev) if dprev is not None else None
    ranks = plan.lno(S, dp, lambda_th=s.get("lambda_th", 0.1), k_min=s.get("k_min", 1), k_max=s.get("k_max", -1),
                     fixed_rank=fixed_rank)
    plan.solve(H, S)
    if mu is None:
        mu, eb, ne = plan.density(s["n_electrons"], s["kT"], D)
    else:
        eb, ne = plan.density_at(mu, s["kT"], D)
    torch.cuda.synchronize()
    out = dict(D=D.cpu().numpy(), mu=mu, e_band=eb, n_e=ne, ranks=ranks)
    if energy:
        E = torch.zeros_like(S)
        out["tr_es"] = plan.energy_density(E)
        torch.cuda.synchronize()
        out["E"] = E.cpu().numpy()
    if keep_plan:
        out["plan"] = plan
        out["dev"] = (H, S, D)
    elif own:
        plan.close()
    return out
