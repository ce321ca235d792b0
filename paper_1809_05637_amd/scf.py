"""Toy self-consistent loop on the device, through the C ABI.

Sec. II.C step (i): the LNOs are recomputed at every SCF step from the density of the step
before.  One step is ldc_potential (H = H0 + (v_i + v_j)/2 S), ldc_lno (from the previous
density; plain DC at the first step unless an initial density is given), ldc_solve,
ldc_density, ldc_mulliken and ldc_scf_mix (linear mixing of the Mulliken populations,
v = U (q_in - q0)).  This module only sequences those calls and owns the device buffers.
"""
from __future__ import annotations

import numpy as np


def scf_loop(plan, H0, S, n_electrons, kT, U, alpha, steps, q0=None, lno=True, lambda_th=0.1, k_min=1, k_max=-1,
             fixed_rank=None, D0=None, keep=False, on_step=None):
    """Runs ``steps`` SCF steps on the plan's stream.  H0, S (and D0): device tensors in the
    block layout.  Returns one record per step: residual, mu, e_band, n_e (and, with keep=True,
    host copies of q_in, q_out and D).  on_step(k, record) is called after every step.  q0 (host
    array) defaults to the library's neutral reference populations (ldc_reference_populations)."""
    import torch
    dev = S.device
    if q0 is None:
        q0_d = torch.empty(plan.n_atoms, dtype=torch.float64, device=dev)
        plan.reference_populations(n_electrons, q0_d)   # neutral atoms at the system's filling
    else:
        q0_d = torch.as_tensor(np.asarray(q0, dtype=np.float64), device=dev)
    q_in = q0_d.clone()
    q_out = torch.zeros_like(q0_d)
    v = torch.zeros_like(q0_d)
    H = torch.empty_like(H0)
    D = torch.zeros_like(S)
    Dprev = D0.clone() if D0 is not None else None
    history = []
    for k in range(steps):
        rec = {}
        if keep:
            rec["q_in"] = q_in.cpu().numpy()
        plan.potential(H0, S, v, H)
        plan.lno(S, Dprev if lno else None, lambda_th=lambda_th, k_min=k_min, k_max=k_max, fixed_rank=fixed_rank,
                 want_ranks=False)
        plan.solve(H, S)
        mu, eb, ne = plan.density(n_electrons, kT, D)
        plan.mulliken(D, S, q_out)
        if keep:
            rec["q_out"] = q_out.cpu().numpy()
            rec["D"] = D.cpu().numpy()
        rec.update(residual=plan.scf_mix(q_out, q_in, q0_d, U, alpha, v), mu=mu, e_band=eb, n_e=ne)
        history.append(rec)
        if on_step is not None:
            on_step(k, rec)
        if Dprev is None:
            Dprev = torch.empty_like(D)
        Dprev, D = D, Dprev
    return history
