"""Conventional O(N^3) density matrix of the whole system (Eq. 2, 8-12), for identity checks.

Loewdin route, independent of the Cholesky-based generalized solver used per cluster:
S = V s V^T, X = S^{-1/2} = V s^{-1/2} V^T; the Loewdin Hamiltonian X H X = Y e Y^T;
rho = X Y f(e) Y^T X (Eq. 12: the Loewdin density is S^{1/2} rho S^{1/2}); mu by
bisection on g sum_mu f(e_mu - mu) = N_e (in the orthonormal basis every weight is 1).
"""
from __future__ import annotations

import numpy as np

from .density import fermi


def dense(sysd, values):
    n_orb = sysd["n_orb"]
    offs = np.concatenate([[0], np.cumsum(n_orb)])
    n = int(offs[-1])
    out = np.zeros((n, n))
    row_ptr, col, blk_off = sysd["row_ptr"], sysd["col"], sysd["blk_off"]
    for i in range(len(n_orb)):
        for b in range(row_ptr[i], row_ptr[i + 1]):
            j = col[b]
            mi, mj = n_orb[i], n_orb[j]
            out[offs[i]: offs[i + 1], offs[j]: offs[j + 1]] = values[blk_off[b]: blk_off[b] + mi * mj].reshape(mi, mj)
    return out, offs


def exact_density(sysd, kT=None, n_electrons=None, g=2.0):
    """Returns (rho dense, mu, eigenvalues)."""
    kT = sysd["kT"] if kT is None else kT
    n_electrons = sysd["n_electrons"] if n_electrons is None else n_electrons
    h, _ = dense(sysd, sysd["H"])
    s, _ = dense(sysd, sysd["S"])
    sv, vv = np.linalg.eigh(s)
    x = (vv * (1.0 / np.sqrt(sv))) @ vv.T
    e, y = np.linalg.eigh(x @ h @ x)
    lo, hi = e[0] - 40 * kT, e[-1] + 40 * kT
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if hi - lo <= 4e-16 * max(1.0, abs(mid)):
            break
        if g * np.sum(fermi((e - mid) / kT)) < n_electrons:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    f = fermi((e - mu) / kT)
    xy = x @ y
    rho = (xy * f) @ xy.T
    return rho, mu, e


def exact_density_blocks(sysd, rho):
    """The exact rho restricted to the BSR pattern, as a flat value array."""
    n_orb = sysd["n_orb"]
    offs = np.concatenate([[0], np.cumsum(n_orb)])
    out = np.zeros_like(sysd["S"])
    row_ptr, col, blk_off = sysd["row_ptr"], sysd["col"], sysd["blk_off"]
    for i in range(len(n_orb)):
        for b in range(row_ptr[i], row_ptr[i + 1]):
            j = col[b]
            mi, mj = n_orb[i], n_orb[j]
            out[blk_off[b]: blk_off[b] + mi * mj] = rho[offs[i]: offs[i + 1], offs[j]: offs[j + 1]].ravel()
    return out
