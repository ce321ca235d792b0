"""Complex-conjugate eigenvalue pairs of Lambda on the GPU (Sec. II.B, Eq. 20-22; reading R1):
the tiny chain whose Lambda matrices have pairs, built through ldc_lno / ldc_solve /
ldc_density and compared with the oracle -- ranks equal, density rows and band energy at the
parity bar -- with the pair kept by the rank rule, cut through by a fixed rank (the cut moves
past the pair) and cut with k_max forbidding that (the cut moves before the pair)."""
import numpy as np
import pytest

import oracle
from gpu_util import gpu_build
from pair_systems import tiny_pair_system

pytestmark = pytest.mark.gpu


def _kept_pairs(s, dprev, ranks):
    """Number of atoms whose kept LNO span includes a complex-conjugate pair."""
    kept = 0
    for j in range(s["n_atoms"]):
        w, _ = oracle.lno.sorted_eig(oracle.lambda_matrix(s, dprev, j))
        kept += int(np.any(w.imag[: int(ranks[j])] != 0))
    return kept


@pytest.mark.parametrize("case", ["rule", "fixed_past", "fixed_before"])
def test_pairs_through_the_abi(case):
    s, dprev = tiny_pair_system()
    s = dict(s)
    fixed = None
    if case != "rule":
        fixed = 2          # atom 1: the cut between its two pair members
        if case == "fixed_before":
            s["k_max"] = 2  # moving past the pair would exceed k_max: the cut moves before it
    ref = oracle.density_build(s, dprev=dprev, fixed_rank=fixed, workers=1)
    got = gpu_build(s, dprev=dprev, fixed_rank=fixed)
    ranks = np.asarray(got["ranks"])
    print(f"[pairs] {case}: ranks gpu {ranks.tolist()} oracle {np.asarray(ref['ranks']).tolist()}", flush=True)
    assert np.array_equal(ranks, np.asarray(ref["ranks"]))
    assert _kept_pairs(s, dprev, ranks) >= 1          # a kept pair runs through the device path
    if case == "fixed_past":
        assert ranks[1] == 3
    if case == "fixed_before":
        assert ranks[1] == 1
    err = float(np.abs(got["D"] - ref["D"]).max())
    de = abs(got["e_band"] - ref["e_band"]) / s["n_atoms"]
    print(f"[pairs] {case}: max|dD|={err:.3e} dE_band/atom={de:.3e}", flush=True)
    assert err <= 1e-9 and de <= 1e-10
