"""Oracle energy density rows (Eq. 25 with Eq. 27) pinned by exact relations.

* whole-system cluster: the exact e = C diag(f eps) C^T satisfies e = rho H S^{-1}
  (C^T H = eps C^T S), an independent route through the exact density and H, S;
* 1D ring: plane waves give e_0j = (1/L) sum_k f(eps_k - mu) eps_k cos(kj),
  eps_k = eps + 2t cos k (the Appendix's model);
* any DC / DC-LNO build: g Tr(E S) = g sum_i sum_mu f eps w = E_band, because F_i lies in the
  short region (the same argument as g Tr(D S) = N_e, Eq. 13).
"""
import numpy as np
import pytest

import oracle
import synth


def test_energy_density_whole_system_equals_rho_h_sinv():
    s = synth.small("sc64_whole")
    r = oracle.density_build(s, energy=True, workers=1)
    rho, mu, e = oracle.exact_density(s)
    h, _ = oracle.exact.dense(s, s["H"])
    sm, _ = oracle.exact.dense(s, s["S"])
    e_ref = oracle.exact_density_blocks(s, rho @ h @ np.linalg.inv(sm))
    assert abs(mu - r["mu"]) < 1e-12
    assert np.abs(r["E"] - e_ref).max() < 1e-11
    # the energy-weighted rows are not the density rows (a dropped eps factor would pass above
    # only if H S^-1 were the identity on the pattern)
    assert np.abs(r["E"] - r["D"]).max() > 1e-2


@pytest.mark.parametrize("n,eps,t", [(32, 0.0, 1.0), (30, 0.3, 0.7)])
def test_energy_density_ring_closed_form(n, eps, t):
    s = synth.ring(n, eps=eps, t=t, kT=0.05)
    s["n_electrons"] = float(n)
    r = oracle.density_build(s, energy=True, workers=1)
    k = 2 * np.pi * np.arange(n) / n
    ek = eps + 2 * t * np.cos(k)
    for i in (0, 7):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            dj = (s["col"][b] - i) % n
            ref = np.mean(oracle.fermi((ek - r["mu"]) / s["kT"]) * ek * np.cos(k * dj))
            assert abs(r["E"][s["blk_off"][b]] - ref) < 1e-13


@pytest.mark.parametrize("name,lno", [("sc27", False), ("dia216", True)])
def test_trace_es_equals_band_energy(name, lno):
    s = synth.small(name)
    r0 = oracle.density_build(s, lno=False, energy=not lno)
    r = r0 if not lno else oracle.density_build(s, dprev=r0["D"], energy=True,
                                                fixed_rank=s["fixed_k"] if s["fixed_k"] >= 0 else None)
    assert abs(r["tr_es"] - r["e_band_spectral"]) < 1e-10 * abs(r["e_band_spectral"])
    assert abs(r["tr_es"] - r["e_band"]) < 1e-10 * abs(r["e_band"])
