"""Truncated cluster and short/long regions of every atom (Sec. III, steps (i)-(iv)).

(i)   cluster C_i: every atom within the sphere of radius r_L around atom i;
(ii)  first neighbouring atoms F_i: atoms with a structurally nonzero overlap block with
      atom i (the row of the S pattern); second neighbouring atoms: the rest of C_i;
(iii) short region: the atoms inside a sphere of radius r_S, where r_S is chosen so the
      sphere holds about N_F + kappa N_S atoms;
(iv)  long region: C_i minus the short region.

Readings where the text is open:
* distances are minimum-image distances on periodic axes; every atom appears once in a
  cluster even when several of its images are inside r_L (Gamma-point supercell);
* the sphere is inclusive (dist <= r_L, with a 1e-9 relative tolerance);
* "as close as possible" is read as the smallest neighbour shell whose cumulative count
  is >= N_F + kappa N_S (the nearest-count rule would give 239 rather than the printed 275
  for the diamond example of Sec. IV.C);
* F_i is always kept in the short region;
* plain DC (no LNOs) puts the whole cluster in the short region.
Cluster order used by the oracle: short atoms by (distance, index) -- the centre first --
then long atoms by (distance, index).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Region:
    center: int
    members: np.ndarray      # atom indices, short first then long
    dist: np.ndarray         # distances of the members
    n_short: int
    n_fna: int               # N_F (includes the centre)
    n_cluster: int           # N_F + N_S

    @property
    def short(self):
        return self.members[: self.n_short]

    @property
    def long(self):
        return self.members[self.n_short:]


def min_image_dist(pos, cell, periodic, i):
    d = pos - pos[i]
    lengths = np.diag(cell)
    for ax in range(3):
        if periodic[ax]:
            d[:, ax] -= lengths[ax] * np.round(d[:, ax] / lengths[ax])
    return np.sqrt((d * d).sum(axis=1))


def plan_regions(sysd, r_L=None, kappa=None, lno=True, shell_tol=1e-8):
    """Regions of every atom.  Returns a list of Region."""
    pos = np.asarray(sysd["pos"], dtype=np.float64)
    cell = np.asarray(sysd["cell"], dtype=np.float64)
    periodic = np.asarray(sysd["periodic"])
    row_ptr, col = sysd["row_ptr"], sysd["col"]
    r_L = sysd["r_L"] if r_L is None else r_L
    kappa = sysd["kappa"] if kappa is None else kappa
    tol = 1e-9 * max(1.0, r_L)
    stol = shell_tol * max(1.0, r_L)
    out = []
    for i in range(len(pos)):
        dist = min_image_dist(pos, cell, periodic, i)
        in_c = np.nonzero(dist <= r_L + tol)[0]
        fna = set(col[row_ptr[i]: row_ptr[i + 1]].tolist())
        fna.add(i)
        order = np.lexsort((in_c, dist[in_c]))
        c_atoms = in_c[order]
        c_dist = dist[c_atoms]
        n_c = len(c_atoms)
        fna_in = [j for j in c_atoms if j in fna]
        missing = fna - set(c_atoms.tolist())
        if missing:
            raise ValueError(f"atom {i}: pattern neighbours outside r_L: {sorted(missing)[:5]}")
        n_f = len(fna_in)
        if not lno:
            out.append(Region(i, c_atoms, c_dist, n_c, n_f, n_c))
            continue
        target = n_f + kappa * (n_c - n_f)
        # shells: maximal runs of equal distance (within tolerance)
        shell_end = []
        for k in range(n_c):
            if k == n_c - 1 or c_dist[k + 1] > c_dist[k] + stol:
                shell_end.append(k + 1)
        n_short_sphere = n_c
        for e in shell_end:
            if e >= target - 1e-12:
                n_short_sphere = e
                break
        short_mask = np.zeros(n_c, dtype=bool)
        short_mask[:n_short_sphere] = True
        for k, j in enumerate(c_atoms):
            if j in fna:
                short_mask[k] = True
        members = np.concatenate([c_atoms[short_mask], c_atoms[~short_mask]])
        mdist = np.concatenate([c_dist[short_mask], c_dist[~short_mask]])
        out.append(Region(i, members, mdist, int(short_mask.sum()), n_f, n_c))
    return out
