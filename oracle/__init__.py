"""CPU FP64 oracle for the DC-LNO density build (Ozaki, Fukuda & Jiang, arXiv 1809.05637).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this package.  It shares no code with the
HIP library: it reads the inputs made by ``synth`` and nothing else.

It is a plain, slow, step-by-step restatement of the method in the paper's order:

* ``regions``  -- truncated cluster of every atom, first/second neighbouring atoms and the
                  short/long split (Sec. III, steps (i)-(iv)).
* ``lno``      -- Lambda matrix (Eq. 17), its nonsymmetric eigendecomposition (Eq. 20) and
                  the low-rank selection lambda >= lambda_th (Eq. 22 and Sec. II.B (i)-(iii)).
* ``cluster``  -- cluster Hamiltonian/overlap with PAO and LNO blocks (Eq. 26), the
                  generalized eigenproblem H c = eps S c, and the atom's spectral weights.
* ``density``  -- common chemical potential by bisection on the electron count (Eq. 13, 16,
                  Sec. II.C step (iv)), density-matrix rows from the spectral Green function
                  (Eq. 24 with Eq. 27, Sec. II.C step (v)), windowed density rows for
                  energy-window LNOs (Sec. II.B), energy density rows (Eq. 25 with
                  Eq. 27), band energy and electron count.
* ``exact``    -- the conventional O(N^3) density matrix of the whole system by the Loewdin
                  route (Eq. 2, 8-12), used for the whole-system identity checks.
* ``driver``   -- ``density_build``: the whole pipeline for one build.
* ``scf``      -- a toy self-consistent loop around the build (LNOs regenerated every step,
                  Sec. II.C (i)): Mulliken populations, a Hubbard-like potential, linear mixing.

Readings of points the paper leaves open are listed in each module's docstring.
Parity status: every function is pinned by tests under tests/test_oracle_*.py (paper
counts, closed forms, identities, brute force in 40-digit arithmetic).
"""
from .regions import plan_regions, Region  # noqa: F401
from .lno import lambda_matrix, lno_basis, select_rank, all_lnos  # noqa: F401
from .cluster import cluster_matrices, solve_cluster  # noqa: F401
from .density import (fermi, bisect_mu, density_rows, energy_density_rows, band_energy_and_count,  # noqa: F401
                      window_weights, window_rows)
from .exact import exact_density, exact_density_blocks  # noqa: F401
from .driver import density_build  # noqa: F401
from .scf import mulliken, potential, reference_populations, scf_loop  # noqa: F401
