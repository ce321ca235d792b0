"""Seeded tiny systems whose Lambda matrices (Eq. 17) have complex-conjugate eigenvalue pairs
(reading R1 of the design notes): shared by the brute-force oracle test and the GPU tests.
Inputs only -- no arithmetic of the method."""
import numpy as np

import synth


def tiny_pair_system():
    """8-atom periodic chain, 3 orbitals per atom, r_L = 3 (every cluster has long atoms), and a
    symmetric "previous density" drawn on the overlap pattern (any rho is allowed for the LNOs):
    Lambda is nonsymmetric with complex pairs on several atoms."""
    s = synth.make_system("sc", (8, 1, 1), (1, 0, 0), 3, lambda rng, sub, m: rng.normal(0, 0.1, (len(sub), m)),
                          1.0, 0.8, 1.0 + 1e-6, 4242)
    n = s["n_atoms"]
    s.update(r_L=3.0, kappa=0.3, kT=0.05, spin_g=2, n_electrons=float(3 * n), lno=True,
             lambda_th=0.1, k_min=1, k_max=-1, fixed_k=-1, name="tiny_pair8")
    rng = np.random.default_rng(15)
    # the nonzero entries of the dense overlap matrix (the onsite blocks are the identity, so
    # their off-diagonal entries stay zero), then a random symmetric matrix on them, back to blocks
    offs = np.concatenate([[0], np.cumsum(s["n_orb"])])
    nb = int(offs[-1])
    mask = np.zeros((nb, nb), dtype=bool)
    for i in range(n):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            o, mi, mj = s["blk_off"][b], s["n_orb"][i], s["n_orb"][j]
            mask[offs[i]:offs[i + 1], offs[j]:offs[j + 1]] = s["S"][o:o + mi * mj].reshape(mi, mj) != 0.0
    x = rng.standard_normal((nb, nb)) * 0.3
    rho = (x + x.T) * mask
    dprev = np.zeros_like(s["S"])
    for i in range(n):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            o, m = s["blk_off"][b], s["n_orb"][i] * s["n_orb"][j]
            dprev[o:o + m] = rho[offs[i]:offs[i + 1], offs[j]:offs[j + 1]].ravel()
    return s, dprev
