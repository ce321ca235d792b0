"""Oracle pinned by exact identities of the method (Eq. 13, 16, 22, 27; Sec. II)."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import synth


@pytest.fixture(scope="module")
def sc27():
    s = synth.small("sc27")
    return s, oracle.density_build(s, workers=1)


@pytest.fixture(scope="module")
def dia():
    s = synth.small("dia216")
    r0 = oracle.density_build(s, lno=False)
    return s, r0


def test_trace_identity_eq16(sc27):
    """Sum of partial traces of Lambda = Tr(rho S) for the oracle's D and for a random
    symmetric rho on the pattern (Eq. 16 holds for any rho)."""
    s, r = sc27
    tr = sum(np.trace(oracle.lambda_matrix(s, r["D"], j)) for j in range(s["n_atoms"]))
    assert abs(tr - np.dot(r["D"], s["S"])) < 1e-11 * abs(tr)
    rng = np.random.default_rng(5)
    rho_d, offs = oracle.exact.dense(s, r["D"])
    x = rng.standard_normal(rho_d.shape)
    mask = (rho_d != 0).astype(float)
    rnd = (x + x.T) * mask
    rvals = oracle.exact_density_blocks(s, rnd)
    tr = sum(np.trace(oracle.lambda_matrix(s, rvals, j)) for j in range(s["n_atoms"]))
    assert abs(tr - np.dot(rvals, s["S"])) < 1e-10 * max(1.0, abs(tr))


def test_electron_count_and_band_energy(sc27):
    """g Tr(D S) = N_e at the bisected mu, and g sum f eps w = g Tr(D H) (Eq. 13 with 27)."""
    s, r = sc27
    assert abs(r["n_e"] - s["n_electrons"]) < 1e-10 * s["n_electrons"]
    assert abs(r["e_band"] - r["e_band_spectral"]) < 1e-10 * abs(r["e_band"])


def test_weights_sum_to_orbital_count(sc27):
    s, r = sc27
    for i, (eps, w) in r["spectra"].items():
        assert abs(w.sum() - s["n_orb"][i]) < 1e-11


def test_whole_system_cluster_is_exact():
    """A cluster equal to the whole system reproduces the conventional diagonalization
    (torus reading): D on the pattern, mu and E_band."""
    s = synth.small("sc64_whole")
    r = oracle.density_build(s)
    assert all(len(reg.members) == s["n_atoms"] for reg in r["regions"])
    rho, mu, e = oracle.exact_density(s)
    ex = oracle.exact_density_blocks(s, rho)
    assert np.abs(ex - r["D"]).max() < 1e-12
    assert abs(mu - r["mu"]) < 1e-12
    g = 2.0
    e_exact = g * np.sum(oracle.fermi((e - mu) / s["kT"]) * e)
    assert abs(e_exact - r["e_band"]) < 1e-10 * abs(e_exact)


def test_full_rank_lno_equals_plain_dc(dia):
    """Keeping every eigenvector of Lambda (Eq. 22 with all terms) gives plain DC."""
    s, r0 = dia
    full = oracle.density_build(s, dprev=r0["D"], fixed_rank=int(s["n_orb"][0]))
    assert np.abs(full["D"] - r0["D"]).max() < 1e-12
    assert abs(full["mu"] - r0["mu"]) < 1e-11


def test_lno_span_invariance(dia):
    """Only the span of the LNOs enters Eq. 27: any invertible k x k change of basis of
    every U_j leaves D unchanged."""
    s, r0 = dia
    regions = oracle.plan_regions(s, lno=True)
    us, _, ranks = oracle.all_lnos(s, r0["D"])
    rng = np.random.default_rng(3)
    us2 = [u @ (np.eye(u.shape[1]) + 0.3 * rng.standard_normal((u.shape[1], u.shape[1]))) for u in us]
    for i in (0, 7, 101):
        a = oracle.solve_cluster(s, regions[i], us, ranks)
        b = oracle.solve_cluster(s, regions[i], us2, ranks)
        assert np.abs(a["eps"] - b["eps"]).max() < 1e-11
        da = oracle.density.density_rows(a["rows"][i], a["rows"], a["eps"], 0.0, s["kT"])
        db = oracle.density.density_rows(b["rows"][i], b["rows"], b["eps"], 0.0, s["kT"])
        for j in da:
            assert np.abs(da[j] - db[j]).max() < 1e-11


def test_lno_basis_properties(dia):
    """U_j is S_jj-orthonormal and spans the kept eigenvectors of Lambda_j (Eq. 20-22)."""
    s, r0 = dia
    for j in (0, 5, 77):
        u, lam_sorted, k = oracle.lno_basis(s, r0["D"], j, 0.1, fixed=4)
        sjj = oracle.lno.block(s, s["S"], j, j)
        assert np.abs(u.T @ sjj @ u - np.eye(k)).max() < 1e-13
        lam = oracle.lambda_matrix(s, r0["D"], j)
        # invariant subspace: Lambda U = U X for some k x k X
        x = np.linalg.lstsq(u, lam @ u, rcond=None)[0]
        assert np.abs(lam @ u - u @ x).max() < 1e-12
        assert np.allclose(np.sort(np.linalg.eigvals(x).real)[::-1], lam_sorted[:k].real, atol=1e-12)


def test_cholesky_route_matches_lowdin_route(dia):
    """Per-cluster spectrum and weights by an independent Loewdin route (S^{-1/2} from the
    eigendecomposition of S) agree with the Cholesky-based generalized solver."""
    s, r0 = dia
    regions = oracle.plan_regions(s, lno=True)
    us, _, ranks = oracle.all_lnos(s, r0["D"])
    for i in (3, 150):
        hc, sc, offs = oracle.cluster_matrices(s, regions[i], us, ranks)
        sv, vv = np.linalg.eigh(sc)
        x = (vv / np.sqrt(sv)) @ vv.T
        e, y = np.linalg.eigh(x @ hc @ x)
        c = x @ y
        m = s["n_orb"][i]
        w = np.sum(c[:m] * (sc[:m] @ c), axis=0)
        ref = oracle.solve_cluster(s, regions[i], us, ranks)
        assert np.abs(e - ref["eps"]).max() < 1e-12
        assert np.abs(w - ref["w"]).max() < 1e-12


def test_idempotency_gapped_exact():
    """D S D = D for the exact density of a gapped system at low temperature: a checkerboard
    simple-cubic lattice with onsite +-0.5 and nearest-neighbour hopping, S = I (gap >= 1)."""
    sysd = synth.make_system("sc", (4, 4, 4), (1, 1, 1), 1, lambda rng, sub, m: np.zeros((64, 1)), 0.1, 1e9,
                             1.0 + 1e-6, 11, s_amp=0.0)
    pos = sysd["pos"]
    parity = (np.round(pos).astype(int).sum(axis=1) % 2)
    for i in range(64):
        b = sysd["row_ptr"][i] + np.searchsorted(sysd["col"][sysd["row_ptr"][i]:sysd["row_ptr"][i + 1]], i)
        sysd["H"][sysd["blk_off"][b]] = 0.5 if parity[i] else -0.5
    sysd.update(kT=0.01, n_electrons=64.0)
    rho, mu, e = oracle.exact_density(sysd)
    s, _ = oracle.exact.dense(sysd, sysd["S"])
    gap = e[32] - e[31]
    assert gap >= 1.0
    assert np.abs(rho @ s @ rho - rho).max() < max(1e-13, np.exp(-gap / (2 * 0.01)))


def test_mu_bisection_brackets():
    spectra = [(np.array([-1.0, 0.0, 1.0]), np.array([1.0, 1.0, 1.0]))]
    mu, it = oracle.bisect_mu(spectra, 3.0, 0.01)
    assert abs(mu) < 1e-12
    with pytest.raises(ValueError):
        oracle.bisect_mu(spectra, 6.0, 0.01)
    with pytest.raises(ValueError):
        oracle.bisect_mu(spectra, 0.0, 0.01)
