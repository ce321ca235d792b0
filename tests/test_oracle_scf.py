"""Oracle toy SCF loop (LNOs regenerated every step, Sec. II.C (i)) pinned by independent routes.

* Mulliken populations of a whole-system cluster (DC = exact diagonalization) against
  g sum_{a in i} (rho S)_aa from the exact density of the Loewdin route;
* a whole-system SCF trajectory against an exact SCF written here with dense matrix algebra
  (H = H0 + (diag(w) S + S diag(w)) / 2, generalized eigh of the whole system, Fermi filling,
  populations from rho S), step by step;
* a uniform potential v shifts every eigenvalue by v: mu moves by v, D is unchanged and
  E_band moves by v N_e, for plain DC and for DC-LNO (the LNOs depend on D_prev and S only).
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth


def _dense(s, vals):
    n_orb = s["n_orb"]
    offs = np.concatenate([[0], np.cumsum(n_orb)])
    out = np.zeros((offs[-1], offs[-1]))
    for i in range(s["n_atoms"]):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            blk = vals[s["blk_off"][b]: s["blk_off"][b] + n_orb[i] * n_orb[j]].reshape(n_orb[i], n_orb[j])
            out[offs[i]: offs[i + 1], offs[j]: offs[j + 1]] += blk
    return out


def _fermi(x):
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def _exact_scf(s, U, alpha, steps):
    g = 2.0
    h0, sm = _dense(s, s["H"]), _dense(s, s["S"])
    n_orb = np.asarray(s["n_orb"])
    atom_of = np.repeat(np.arange(s["n_atoms"]), n_orb)
    q0 = s["n_electrons"] * n_orb / n_orb.sum()
    q_in = q0.copy()
    out = []
    for _ in range(steps):
        w = (U * (q_in - q0))[atom_of]
        h = h0 + 0.5 * (w[:, None] * sm + sm * w[None, :])
        e, c = scipy.linalg.eigh(h, sm)
        lo, hi = e[0] - 40 * s["kT"], e[-1] + 40 * s["kT"]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if hi - lo <= 4e-16 * max(1.0, abs(mid)):
                break
            if g * np.sum(_fermi((e - mid) / s["kT"])) < s["n_electrons"]:
                lo = mid
            else:
                hi = mid
        mu = 0.5 * (lo + hi)
        rho = (c * _fermi((e - mu) / s["kT"])) @ c.T
        q_out = g * np.bincount(atom_of, weights=np.diag(rho @ sm))
        out.append(dict(q_in=q_in.copy(), q_out=q_out, mu=mu))
        q_in = q_in + alpha * (q_out - q_in)
    return out


def test_mulliken_whole_system_equals_rho_s_diagonal():
    s = synth.small("sc64_whole")
    r = oracle.density_build(s, workers=1)
    rho, mu, _ = oracle.exact_density(s)
    sm = _dense(s, s["S"])
    atom_of = np.repeat(np.arange(s["n_atoms"]), s["n_orb"])
    q_ref = 2.0 * np.bincount(atom_of, weights=np.diag(rho @ sm))
    q = oracle.mulliken(s, r["D"])
    assert np.abs(q - q_ref).max() < 1e-11
    assert abs(q.sum() - s["n_electrons"]) < 1e-9
    # not uniform: a partition error that kept the total would still show here
    assert q.max() - q.min() > 1e-3


def test_scf_whole_system_follows_exact_scf():
    s = synth.small("sc64_whole")
    U, alpha, steps = 0.5, 0.4, 6
    hist = oracle.scf_loop(s, U, alpha, steps, lno=False, workers=1)
    ref = _exact_scf(s, U, alpha, steps)
    for k in range(steps):
        assert np.abs(hist[k]["q_in"] - ref[k]["q_in"]).max() < 1e-10, k
        assert np.abs(hist[k]["q_out"] - ref[k]["q_out"]).max() < 1e-10, k
        assert abs(hist[k]["mu"] - ref[k]["mu"]) < 1e-11, k
    # the potential does act: the populations move between steps and the loop contracts
    assert np.abs(hist[1]["q_out"] - hist[0]["q_out"]).max() > 1e-4
    assert hist[-1]["residual"] < 0.5 * hist[1]["residual"]


@pytest.mark.parametrize("name", ["sc27", "dia216"])
def test_uniform_potential_shifts_the_spectrum(name):
    s = synth.small(name)
    c = 0.37
    dprev = None
    fixed = None
    if s.get("lno"):
        dprev = oracle.density_build(s)["D"]
        fixed = int(s["fixed_k"]) if int(s.get("fixed_k", -1)) >= 0 else None
    r0 = oracle.density_build(s, dprev=dprev, fixed_rank=fixed)
    h = oracle.potential(s, s["H"], np.full(s["n_atoms"], c))
    r1 = oracle.density_build(dict(s, H=h), dprev=dprev, fixed_rank=fixed)
    assert abs(r1["mu"] - (r0["mu"] + c)) < 1e-11
    assert np.abs(r1["D"] - r0["D"]).max() < 1e-10
    assert abs(r1["e_band"] - (r0["e_band"] + c * r0["n_e"])) < 1e-8 * max(1.0, abs(r0["e_band"]))


def test_reference_populations_are_neutral():
    s = synth.small("fcc_slab")
    q0 = oracle.reference_populations(s)
    assert abs(q0.sum() - s["n_electrons"]) < 1e-9
    assert np.allclose(q0 / np.asarray(s["n_orb"]), s["n_electrons"] / np.sum(s["n_orb"]))
