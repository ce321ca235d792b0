"""Localized natural orbitals (Sec. II.B).

For every atom j:
(i)   Lambda_j = sum_k rho_{jk} S_{kj}  (Eq. 17; k runs over the structural overlap
      neighbours of j, the sum over images already folded into the Gamma-point blocks);
(ii)  the nonsymmetric eigendecomposition V^{-1} Lambda_j V = lambda (Eq. 20), done with
      LAPACK's general eigensolver (numpy.linalg.eig);
(iii) keep the eigenvectors whose eigenvalue is >= lambda_th (Eq. 22).

Readings where the text is open:
* eigenvalues are ranked by their real part, descending, ties by column index; a
  complex-conjugate pair is kept or dropped as a whole and contributes the real and
  imaginary parts of one member as two real basis vectors;
* rank rule: k = clamp(#{Re lambda >= lambda_th}, k_min, k_max); a fixed rank per atom
  overrides the count (used to pin discrete choices in parity runs);
* only the span of the kept vectors enters the cluster problem (Eq. 27 is invariant under
  an invertible change of basis inside the span), so the kept real basis B is made
  S_jj-orthonormal by the Loewdin map B (B^T S_jj B)^{-1/2}, which keeps the span.
"""
from __future__ import annotations

import numpy as np


def block(sysd, values, i, j):
    """Block (i, j) of a BSR value array, or None if (i, j) is outside the pattern."""
    row_ptr, col, blk_off, n_orb = sysd["row_ptr"], sysd["col"], sysd["blk_off"], sysd["n_orb"]
    lo, hi = row_ptr[i], row_ptr[i + 1]
    k = lo + np.searchsorted(col[lo:hi], j)
    if k >= hi or col[k] != j:
        return None
    mi, mj = n_orb[i], n_orb[j]
    return values[blk_off[k]: blk_off[k] + mi * mj].reshape(mi, mj)


def lambda_matrix(sysd, dprev, j):
    """Eq. 17: Lambda_j = sum_k rho_{jk} S_{kj}, an M_j x M_j nonsymmetric matrix."""
    row_ptr, col = sysd["row_ptr"], sysd["col"]
    m = sysd["n_orb"][j]
    lam = np.zeros((m, m))
    for b in range(row_ptr[j], row_ptr[j + 1]):
        k = col[b]
        lam += block(sysd, dprev, j, k) @ block(sysd, sysd["S"], k, j)
    return lam


def sorted_eig(lam):
    """Eigenpairs of Lambda ranked by real part, descending (stable on ties)."""
    w, v = np.linalg.eig(lam)
    order = np.argsort(-w.real, kind="stable")
    return w[order], v[:, order]


def select_rank(eigvals, lambda_th, k_min=1, k_max=-1, fixed=None):
    """Number of kept LNOs for eigenvalues already ranked by real part (descending).

    k = clamp(#{Re lambda >= lambda_th}, k_min, k_max), or ``fixed`` if given; a cut
    through a complex-conjugate pair moves past the pair (or before it if that would
    exceed k_max)."""
    m = len(eigvals)
    if k_max is None or k_max < 0:
        k_max = m
    if fixed is not None and fixed >= 0:
        k = int(fixed)
    else:
        k = int(np.sum(np.real(eigvals) >= lambda_th))
        k = max(k_min, min(k_max, k))
    k = max(0, min(m, k))
    if 0 < k < m and abs(np.imag(eigvals[k - 1])) > 0 and np.isclose(eigvals[k - 1], np.conj(eigvals[k])):
        k = k + 1 if k + 1 <= k_max else k - 1
    return k


def real_basis(eigvals, eigvecs, k):
    """Real basis of the span of the first k ranked eigenvectors."""
    cols = []
    t = 0
    while t < k:
        if abs(eigvals[t].imag) > 0 and t + 1 < k:
            cols.append(eigvecs[:, t].real)
            cols.append(eigvecs[:, t].imag)
            t += 2
        else:
            cols.append(eigvecs[:, t].real)
            t += 1
    return np.array(cols).T if cols else np.zeros((eigvecs.shape[0], 0))


def lowdin(basis, s_jj):
    """basis (basis^T S_jj basis)^{-1/2}: an S_jj-orthonormal basis of the same span."""
    if basis.shape[1] == 0:
        return basis
    g = basis.T @ s_jj @ basis
    e, u = np.linalg.eigh(g)
    return basis @ (u * (1.0 / np.sqrt(e))) @ u.T


def lno_basis(sysd, dprev, j, lambda_th, k_min=1, k_max=-1, fixed=None):
    """LNOs of atom j: (U_j (M_j x k_j), ranked eigenvalues, k_j)."""
    lam = lambda_matrix(sysd, dprev, j)
    w, v = sorted_eig(lam)
    k = select_rank(w, lambda_th, k_min, k_max, fixed)
    b = real_basis(w, v, k)
    u = lowdin(b, block(sysd, sysd["S"], j, j))
    return u, w, k


def all_lnos(sysd, dprev, lambda_th=None, k_min=None, k_max=None, fixed_rank=None):
    """LNOs of every atom.  ``fixed_rank``: None, an int for all atoms, or an array."""
    lambda_th = sysd["lambda_th"] if lambda_th is None else lambda_th
    k_min = sysd["k_min"] if k_min is None else k_min
    k_max = sysd["k_max"] if k_max is None else k_max
    if fixed_rank is None and sysd.get("fixed_k", -1) >= 0:
        fixed_rank = sysd["fixed_k"]
    n = sysd["n_atoms"]
    us, lams, ranks = [], [], np.zeros(n, dtype=np.int32)
    for j in range(n):
        fx = None
        if fixed_rank is not None:
            fx = int(fixed_rank) if np.isscalar(fixed_rank) else int(fixed_rank[j])
        u, w, k = lno_basis(sysd, dprev, j, lambda_th, k_min, k_max, fx)
        us.append(u)
        lams.append(w)
        ranks[j] = k
    return us, lams, ranks
