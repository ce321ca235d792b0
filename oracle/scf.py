"""Toy self-consistent loop around the DC-LNO density build.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II.C, step (i): the LNOs are recomputed at every SCF step from the density of the step
before, so they become self-consistent with the density.  The paper's SCF needs a DFT
Hamiltonian; this toy replaces it by a Hubbard-like Mulliken potential.  Readings (not in
the paper):

* Mulliken population of atom i from its own density rows (row i of D comes from cluster i):
  q_i = g sum_{j in the pattern row of i} sum_ab D_ij[a, b] S_ij[a, b]
  (with the full density matrix this is g sum_{a in i} (D S)_aa, since S vanishes outside
  the pattern);
* potential v_i = U (q_i^in - q0_i) with reference populations q0_i = N_e M_i / sum_j M_j;
* Hamiltonian H_ij = H0_ij + (v_i + v_j) / 2 S_ij (a uniform v shifts every eigenvalue of
  H c = eps S c by v);
* linear mixing of the input populations, q^in <- q^in + alpha (q^out - q^in).

Step k: H_k from q^in_k; LNOs from D_{k-1} (for k = 0 from the given initial density, or
plain DC without one); one density build (Sec. II.C (i)-(v)); q^out_k; residual
max_i |q^out_k - q^in_k|; then the mixing.  q^in_0 = q0.
"""
from __future__ import annotations

import numpy as np

from .driver import density_build


def mulliken(sysd, dvals, g=None):
    """Mulliken populations of every atom from the density rows ``dvals`` (BSR values)."""
    g = float(sysd.get("spin_g", 2)) if g is None else float(g)
    row_ptr, blk_off = sysd["row_ptr"], sysd["blk_off"]
    prod = dvals * sysd["S"]
    q = np.zeros(sysd["n_atoms"])
    for i in range(sysd["n_atoms"]):
        lo = blk_off[row_ptr[i]]
        hi = blk_off[row_ptr[i + 1]] if row_ptr[i + 1] < len(blk_off) else len(prod)
        q[i] = g * float(np.sum(prod[lo:hi]))
    return q


def potential(sysd, h0, v):
    """H_ij = H0_ij + (v_i + v_j) / 2 S_ij on every pattern block (BSR values)."""
    row_ptr, col, blk_off, n_orb = sysd["row_ptr"], sysd["col"], sysd["blk_off"], sysd["n_orb"]
    h = np.array(h0, dtype=np.float64, copy=True)
    s = sysd["S"]
    for i in range(sysd["n_atoms"]):
        for b in range(row_ptr[i], row_ptr[i + 1]):
            j = int(col[b])
            lo, hi = blk_off[b], blk_off[b] + n_orb[i] * n_orb[j]
            h[lo:hi] += 0.5 * (v[i] + v[j]) * s[lo:hi]
    return h


def reference_populations(sysd):
    """q0_i = N_e M_i / sum_j M_j (neutral atoms at the system's filling)."""
    m = np.asarray(sysd["n_orb"], dtype=np.float64)
    return float(sysd["n_electrons"]) * m / float(m.sum())


def scf_loop(sysd, U, alpha, steps, q0=None, d0=None, lno=None, fixed_rank=None, workers=None):
    """Runs ``steps`` SCF steps; returns one record per step (q_in, q_out, residual, mu,
    e_band, n_e, D and the input H of that step)."""
    if q0 is None:
        q0 = reference_populations(sysd)
    q_in = np.array(q0, dtype=np.float64, copy=True)
    h0 = sysd["H"]
    dprev = d0
    use_lno = bool(sysd.get("lno", True)) if lno is None else bool(lno)
    fixed = fixed_rank
    if fixed is None and int(sysd.get("fixed_k", -1)) >= 0:
        fixed = int(sysd["fixed_k"])
    history = []
    for _ in range(steps):
        v = U * (q_in - q0)
        h = potential(sysd, h0, v)
        s_k = dict(sysd, H=h)
        r = density_build(s_k, dprev=dprev if use_lno else None, fixed_rank=fixed, workers=workers,
                          lno=use_lno and dprev is not None)
        q_out = mulliken(sysd, r["D"])
        res = float(np.max(np.abs(q_out - q_in)))
        history.append(dict(q_in=q_in.copy(), q_out=q_out, residual=res, mu=r["mu"], e_band=r["e_band"],
                            n_e=r["n_e"], D=r["D"], H=h))
        q_in = q_in + alpha * (q_out - q_in)
        dprev = r["D"]
    return history
