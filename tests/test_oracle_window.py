"""Oracle energy-window density rows (the projector of Sec. II.B with another window than the
occupied states) pinned by exact relations.

* the open window (-inf, mu) is the Fermi density itself: W = D;
* the full window (-inf, inf) on a whole-system cluster is C C^T = S^{-1} (from C^T S C = I);
* a finite window on a whole-system cluster equals the windowed density of the Loewdin route
  (S^{-1/2} Y diag(w) Y^T S^{-1/2}, Y the eigenvectors of S^{-1/2} H S^{-1/2}), written here;
* for any build the window above mu and the density add up to the full window (weights
  (1 - f) + f = 1), and g Tr(W S) is the window's state count g sum_i sum_mu w(eps) w_mu;
* on a whole-system cluster Lambda of the unoccupied window is I - Lambda of the density
  (Eq. 17 with S^{-1} S = I), and on the gapped diamond the unoccupied window selects exactly
  the 4 orbitals per atom above the gap as LNOs.
"""
import numpy as np

import oracle
import synth
from oracle.lno import lambda_matrix


def _dense(s, vals):
    n_orb = s["n_orb"]
    offs = np.concatenate([[0], np.cumsum(n_orb)])
    out = np.zeros((offs[-1], offs[-1]))
    for i in range(s["n_atoms"]):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            blk = vals[s["blk_off"][b]: s["blk_off"][b] + n_orb[i] * n_orb[j]].reshape(n_orb[i], n_orb[j])
            out[offs[i]: offs[i + 1], offs[j]: offs[j + 1]] += blk
    return out, offs


def _on_pattern(s, dense, offs):
    out = np.zeros_like(s["S"])
    n_orb = s["n_orb"]
    for i in range(s["n_atoms"]):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            out[s["blk_off"][b]: s["blk_off"][b] + n_orb[i] * n_orb[j]] = \
                dense[offs[i]: offs[i + 1], offs[j]: offs[j + 1]].ravel()
    return out


def test_open_window_below_mu_is_the_density():
    s = synth.small("sc27")
    r = oracle.density_build(s, workers=1)
    w = oracle.density_build(s, mu=r["mu"], window=(-1e6, r["mu"], s["kT"]), workers=1)
    assert np.abs(w["W"] - r["D"]).max() < 1e-15


def test_full_window_whole_system_is_s_inverse():
    s = synth.small("sc64_whole")
    r = oracle.density_build(s, window=(-1e6, 1e6, s["kT"]), workers=1)
    sm, offs = _dense(s, s["S"])
    ref = _on_pattern(s, np.linalg.inv(sm), offs)
    assert np.abs(r["W"] - ref).max() < 1e-11


def test_finite_window_whole_system_matches_loewdin_route():
    s = synth.small("sc64_whole")
    r0 = oracle.density_build(s, workers=1)
    e_lo, e_hi, kT = r0["mu"] - 0.3, r0["mu"] + 0.2, 0.02
    r = oracle.density_build(s, window=(e_lo, e_hi, kT), workers=1)
    h, offs = _dense(s, s["H"])
    sm, _ = _dense(s, s["S"])
    sv, vv = np.linalg.eigh(sm)
    x = (vv / np.sqrt(sv)) @ vv.T
    e, y = np.linalg.eigh(x @ h @ x)
    f = lambda t: 0.5 * (1.0 - np.tanh(0.5 * t))  # noqa: E731
    wt = f((e - e_hi) / kT) - f((e - e_lo) / kT)
    xy = x @ y
    ref = _on_pattern(s, (xy * wt) @ xy.T, offs)
    assert np.abs(r["W"] - ref).max() < 1e-11
    assert 1.0 < r["window_count"] < s["n_electrons"]


def test_windows_add_up_and_count_states():
    s = synth.small("fcc_slab")
    r0 = oracle.density_build(s)
    mu = r0["mu"]
    d1 = oracle.density_build(s, dprev=r0["D"], window=(mu, 1e6, s["kT"]))
    full = oracle.density_build(s, dprev=r0["D"], mu=d1["mu"], window=(-1e6, 1e6, s["kT"]))
    above = oracle.density_build(s, dprev=r0["D"], mu=d1["mu"], window=(d1["mu"], 1e6, s["kT"]))
    assert np.abs(above["W"] + above["D"] - full["W"]).max() < 1e-12
    for r in (d1, full):
        assert abs(r["tr_ws"] - r["window_count"]) < 1e-9 * max(1.0, r["window_count"])


def test_unoccupied_window_lambda_complements_the_density():
    s = synth.small("sc64_whole")
    r = oracle.density_build(s, workers=1)
    mu = r["mu"]
    w = oracle.density_build(s, mu=mu, window=(mu, 1e6, s["kT"]), workers=1)
    for j in (0, 17, 63):
        lam_w = lambda_matrix(s, w["W"], j)
        lam_d = lambda_matrix(s, w["D"], j)
        assert np.abs(lam_w + lam_d - np.eye(s["n_orb"][j])).max() < 1e-11


def test_unoccupied_window_lnos_of_the_gapped_diamond():
    s = synth.small("dia216")
    r = oracle.density_build(s)
    w = oracle.density_build(s, mu=r["mu"], window=(r["mu"], 1e6, s["kT"]))
    _, _, ranks = oracle.all_lnos(s, w["W"], lambda_th=0.5, k_min=1, k_max=-1)
    assert np.all(np.asarray(ranks) == 4)
