"""Common chemical potential, density rows and energy density rows (Sec. II.C steps
(iv)-(v); Eq. 13, 16, 24, 25, 27).

Readings where the text is open (the paper defers the mu search to earlier work):
* Fermi-Dirac occupation f(x) = 1/(1+exp(x)) with x = (eps - mu)/kT, evaluated as
  0.5*(1 - tanh(x/2)) so it never overflows;
* the electron count at chemical potential mu is N(mu) = g sum_i sum_mu f w^(i)_mu with
  spin factor g = 2 (Eq. 13) and the per-atom weights of the cluster problems (Eq. 16);
* bisection from the bracket [min eps - 40 kT, max eps + 40 kT]: mid = (lo + hi)/2; if
  N(mid) < N_e then lo = mid else hi = mid; stop when hi - lo <= 4e-16 max(1, |mid|) or
  after 200 halvings; mu = (lo + hi)/2;
* D is the per-spin density matrix: row block (i, j) comes from cluster i only, for every j
  in the overlap pattern of i (Sec. II.C); it is not symmetrised.
* energy window (Sec. II.B: the projector may select another energy window than the occupied
  states): the smooth box w(eps) = f((eps - e_hi)/kT) - f((eps - e_lo)/kT), the states
  between e_lo and e_hi with Fermi-Dirac edges of width kT; its rows W_ij = C_i diag(w) C_j^T
  take the place of the density for the LNOs.
"""
from __future__ import annotations

import numpy as np


def fermi(x):
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def electron_count(mu, spectra, kT, g=2.0):
    tot = 0.0
    for eps, w in spectra:
        tot += np.sum(fermi((eps - mu) / kT) * w)
    return g * tot


def bisect_mu(spectra, n_electrons, kT, g=2.0, max_iter=200):
    """Bisection for N(mu) = n_electrons.  Returns (mu, iterations)."""
    eps_all = np.concatenate([e for e, _ in spectra])
    w_all = np.concatenate([w for _, w in spectra])
    total = g * np.sum(w_all)
    if not (0.0 < n_electrons < total):
        raise ValueError(f"electron count {n_electrons} outside (0, {total})")
    lo = float(eps_all.min()) - 40.0 * kT
    hi = float(eps_all.max()) + 40.0 * kT
    it = 0
    while it < max_iter:
        mid = 0.5 * (lo + hi)
        if hi - lo <= 4e-16 * max(1.0, abs(mid)):
            break
        n = g * np.sum(fermi((eps_all - mid) / kT) * w_all)
        if n < n_electrons:
            lo = mid
        else:
            hi = mid
        it += 1
    return 0.5 * (lo + hi), it


def density_rows(rows_center, rows, eps, mu, kT):
    """Eq. 24 with Eq. 27: D_{ij} = C_i diag(f) C_j^T for every j in ``rows``."""
    f = fermi((eps - mu) / kT)
    ci = rows_center * f[None, :]
    return {j: ci @ cj.T for j, cj in rows.items()}


def window_weights(eps, e_lo, e_hi, kT):
    """The energy window of the projector: f((eps - e_hi)/kT) - f((eps - e_lo)/kT)."""
    return fermi((eps - e_hi) / kT) - fermi((eps - e_lo) / kT)


def window_rows(rows_center, rows, eps, e_lo, e_hi, kT):
    """Windowed density rows W_ij = C_i diag(w) C_j^T for every j in ``rows``."""
    ci = rows_center * window_weights(eps, e_lo, e_hi, kT)[None, :]
    return {j: ci @ cj.T for j, cj in rows.items()}


def energy_density_rows(rows_center, rows, eps, mu, kT):
    """Eq. 25 with Eq. 27: the energy-weighted integral of the spectral Green function of
    cluster i gives e_{ij} = C_i diag(f eps) C_j^T for every j in ``rows``."""
    fe = fermi((eps - mu) / kT) * eps
    ci = rows_center * fe[None, :]
    return {j: ci @ cj.T for j, cj in rows.items()}


def band_energy_and_count(sysd, dvals, g=2.0):
    """E_band = g sum_ij tr(D_ij H_ji), N_e = g sum_ij tr(D_ij S_ji) over the D pattern.

    With one pattern for H, S and D, tr(D_ij X_ji) = sum(D_ij * X_ij) since X_ji = X_ij^T."""
    return g * float(np.dot(dvals, sysd["H"])), g * float(np.dot(dvals, sysd["S"]))
