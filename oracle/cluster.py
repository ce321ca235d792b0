"""Cluster problem of one atom (Sec. II.C, Eq. 26-27).

The cluster matrices are H^(i) = T^T H_c T and S^(i) = T^T S_c T, where H_c, S_c are the
PAO matrices of the cluster atoms (blocks of the global matrices) and
T = blockdiag(I_{M_j} for short atoms, U_j for long atoms): PAO-PAO, PAO-LNO and LNO-LNO
blocks as in Eq. 26.  The generalized eigenproblem H^(i) c = eps S^(i) c (Sec. II.C step
(iii)) is solved with LAPACK's divide-and-conquer generalized symmetric solver.

The spectral weights of the centre atom i, w_mu = sum_{alpha in i} c_{i alpha, mu}
(S^(i) c_mu)_{i alpha}, give the atom's share of the electron count (the partial trace of
Eq. 16 evaluated with the cluster's eigenpairs): N_i(mu) = sum_mu f(eps_mu) w_mu.
The density rows of atom i follow from the spectral Green function Eq. 27 inserted into
Eq. 24: rho_{i alpha, j beta} = sum_mu f(eps_mu) c_{i alpha, mu} c_{j beta, mu}.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from .lno import block


def member_dims(sysd, region, ranks=None):
    n_orb = sysd["n_orb"]
    dims = []
    for t, j in enumerate(region.members):
        if t < region.n_short or ranks is None:
            dims.append(int(n_orb[j]))
        else:
            dims.append(int(ranks[j]))
    return np.array(dims, dtype=np.int64)


def cluster_matrices(sysd, region, us=None, ranks=None, H=None, S=None):
    """Dense H^(i), S^(i) (Eq. 26) and the member offsets in the reduced basis."""
    H = sysd["H"] if H is None else H
    S = sysd["S"] if S is None else S
    use_lno = us is not None and region.n_short < len(region.members)
    dims = member_dims(sysd, region, ranks if use_lno else None)
    offs = np.concatenate([[0], np.cumsum(dims)])
    d = int(offs[-1])
    hc = np.zeros((d, d))
    sc = np.zeros((d, d))
    mem = region.members
    for a, ja in enumerate(mem):
        ta = None if (a < region.n_short or not use_lno) else us[ja]
        for b, jb in enumerate(mem):
            hb = block(sysd, H, ja, jb)
            if hb is None:
                continue
            sb = block(sysd, S, ja, jb)
            tb = None if (b < region.n_short or not use_lno) else us[jb]
            if ta is not None:
                hb = ta.T @ hb
                sb = ta.T @ sb
            if tb is not None:
                hb = hb @ tb
                sb = sb @ tb
            hc[offs[a]: offs[a + 1], offs[b]: offs[b + 1]] = hb
            sc[offs[a]: offs[a + 1], offs[b]: offs[b + 1]] = sb
    return hc, sc, offs


def solve_cluster(sysd, region, us=None, ranks=None, keep_rows=True):
    """Eigenpairs of the cluster problem of ``region.center``.

    Returns dict(eps (d,), w (d,), dim, rows) where rows maps every first-neighbour atom j
    (the centre included) to the coefficient rows c_{j beta, :} (M_j x d) when keep_rows.
    """
    hc, sc, offs = cluster_matrices(sysd, region, us, ranks)
    eps, c = sl.eigh(hc, sc, driver="gvd")
    m0 = int(sysd["n_orb"][region.center])
    assert region.members[0] == region.center
    sc_c = sc[:m0, :] @ c
    w = np.sum(c[:m0, :] * sc_c, axis=0)
    out = dict(eps=eps, w=w, dim=hc.shape[0])
    if keep_rows:
        row_ptr, col = sysd["row_ptr"], sysd["col"]
        pos = {int(j): t for t, j in enumerate(region.members)}
        rows = {}
        for bidx in range(row_ptr[region.center], row_ptr[region.center + 1]):
            j = int(col[bidx])
            t = pos[j]
            assert t < region.n_short
            rows[j] = c[offs[t]: offs[t + 1], :]
        out["rows"] = rows
    return out


def green(eps, c_i, c_j, z):
    """Eq. 27: G_{i alpha, j beta}(Z) = sum_mu c_{i alpha, mu} c_{j beta, mu} / (Z - eps_mu)."""
    return (c_i * (1.0 / (z - eps))[None, :]) @ c_j.T
