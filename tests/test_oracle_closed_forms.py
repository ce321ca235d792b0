"""Oracle pinned by closed forms: the 1D tight-binding ring (Appendix, Eq. A1-A12)."""
import numpy as np
import pytest

import oracle
import synth


def _ring_fermi_rho(n, eps, t, mu, kT, j):
    k = 2 * np.pi * np.arange(n) / n
    return np.mean(oracle.fermi((eps + 2 * t * np.cos(k) - mu) / kT) * np.cos(k * j))


@pytest.mark.parametrize("n,eps,t", [(32, 0.0, 1.0), (30, 0.3, 0.7)])
def test_ring_density_closed_form(n, eps, t):
    """Whole-ring cluster: plane waves diagonalize H, so
    rho_0j = (1/L) sum_k f(eps + 2t cos k - mu) cos(kj); at half filling the spectrum is
    symmetric about eps, so mu = eps."""
    s = synth.ring(n, eps=eps, t=t, kT=0.05)
    s["n_electrons"] = float(n)
    r = oracle.density_build(s, workers=1)
    assert abs(r["mu"] - eps) < 1e-12
    for i in (0, 5):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            dj = (j - i) % n
            ref = _ring_fermi_rho(n, eps, t, r["mu"], s["kT"], dj)
            assert abs(r["D"][s["blk_off"][b]] - ref) < 1e-13


def _ring_green(n, sites, z):
    s = synth.ring(n, eps=0.0, t=1.0)
    reg = oracle.plan_regions(s, lno=False)[0]
    sol = oracle.solve_cluster(s, reg)
    c0 = sol["rows"][0]
    # coefficient rows of farther sites from the full eigenvector set
    hc, sc, offs = oracle.cluster_matrices(s, reg)
    import scipy.linalg as sl
    eps, c = sl.eigh(hc, sc)
    pos = {int(a): t for t, a in enumerate(reg.members)}
    return [oracle.cluster.green(eps, c[[pos[0]]], c[[pos[j % n]]], z)[0, 0] for j in sites]


@pytest.mark.parametrize("zval", [3.0 + 0.5j, -2.6 + 0.1j, 0.4 + 2.5j])
def test_green_function_appendix(zval):
    """Eq. A2-A6: G00 = 1/sqrt((Z-eps)^2-4t^2) and G01..G04 in terms of G00 and gamma,
    for Z away from the band (the ring of 200 sites equals the infinite chain there)."""
    t = 1.0
    g = _ring_green(200, [0, 1, 2, 3, 4], zval)
    gam = zval / t
    root = np.sqrt(zval * zval - 4 * t * t)
    # branch with G00 ~ 1/Z at large |Z|
    g00 = 1.0 / root if abs(1.0 / root - 1.0 / zval) < abs(-1.0 / root - 1.0 / zval) else -1.0 / root
    ref = [g00,
           g00 * gam / 2 - 1 / (2 * t),
           g00 * (gam ** 2 / 2 - 1) - gam / (2 * t),
           g00 * (gam ** 3 / 2 - 1.5 * gam) - (gam ** 2 - 1) / (2 * t),
           g00 * (gam ** 4 / 2 - 2 * gam ** 2 + 1) - (gam ** 3 - 2 * gam) / (2 * t)]
    for a, b in zip(g, ref):
        assert abs(a - b) < 1e-12


def test_matsubara_sum_matches_spectral_density():
    """Eq. A12: rho_0j = delta_0j/2 + Im[(2i/beta) sum_p G_0j(alpha_p)], alpha_p on the
    Matsubara poles; evaluated with Eq. 27 it converges to the Fermi-weighted density."""
    n, kT = 24, 0.2
    s = synth.ring(n, eps=0.0, t=1.0, kT=kT)
    s["n_electrons"] = float(n)
    r = oracle.density_build(s, workers=1)
    reg = r["regions"][0]
    hc, sc, _ = oracle.cluster_matrices(s, reg)
    import scipy.linalg as sl
    eps, c = sl.eigh(hc, sc)
    pos = {int(a): t for t, a in enumerate(reg.members)}
    beta = 1.0 / kT
    p = np.arange(1, 400001)
    alpha = r["mu"] + 1j * (2 * p - 1) * np.pi / beta
    for j in (0, 1, n - 1):
        cj = c[pos[j]]
        c0 = c[pos[0]]
        amp = c0 * cj
        gsum = np.sum(amp[None, :] / (alpha[:, None] - eps[None, :]))
        rho = (0.5 if j == 0 else 0.0) + np.imag(2j / beta * gsum)
        b = s["row_ptr"][0] + np.searchsorted(s["col"][s["row_ptr"][0]:s["row_ptr"][1]], j)
        assert abs(rho - r["D"][s["blk_off"][b]]) < 2e-5


def _chain_error(dimer, r_L, n=120, kT=0.02):
    s = synth.ring(n, eps=0.0, t=1.0, kT=kT, dimer=dimer, r_L=float(n // 2))
    s["n_electrons"] = float(n)
    exact = oracle.density_build(s)
    s2 = dict(s)
    s2["r_L"] = r_L
    trunc = oracle.density_build(s2)
    return abs(trunc["e_band"] - exact["e_band"]) / n


def test_truncation_gapped_vs_metal():
    """Appendix: for a gapped (dimerized) chain the truncation error of the band energy
    decays quickly with r_L; for the half-filled metallic chain at low T it does not."""
    gap_err = [_chain_error(0.6, r) for r in (4.0, 8.0, 16.0)]
    metal_err = [_chain_error(0.0, r) for r in (4.0, 8.0, 16.0)]
    assert gap_err[2] < 1e-3 * gap_err[0]
    assert gap_err[1] < gap_err[0] and gap_err[2] < gap_err[1]
    assert metal_err[2] > 1e-2 * metal_err[0]
