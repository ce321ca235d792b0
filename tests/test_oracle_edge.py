"""Oracle on the edge-case systems (ragged orbital counts, one-atom clusters, near-maximal
cluster dimension), pinned by closed forms and identities.

* isolated atoms (no bonds, S = I, diagonal H): every cluster is its own atom, so the density
  rows are diag f((h_aa - mu)/kT) and g sum f = N_e at the bisection's mu;
* ragged blocks (1..16 orbitals per atom) and the 912-dimensional clusters: g Tr(D S) = N_e
  (Eq. 13 with F_i inside the short region), and D_ij = D_ji^T does not hold in general (rows
  from different clusters) but the diagonal blocks are symmetric.
"""
import numpy as np

import oracle
import synth


def _fermi(x):
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def test_isolated_atoms_closed_form():
    s = synth.small("isolated")
    r = oracle.density_build(s, workers=1)
    mu, kT = r["mu"], s["kT"]
    n_e = 0.0
    for i in range(s["n_atoms"]):
        b = s["row_ptr"][i]
        assert s["row_ptr"][i + 1] - b == 1 and s["col"][b] == i  # only the diagonal block
        m = s["n_orb"][i]
        o = s["blk_off"][b]
        h = s["H"][o: o + m * m].reshape(m, m)
        f = _fermi((np.diag(h) - mu) / kT)
        assert np.abs(r["D"][o: o + m * m].reshape(m, m) - np.diag(f)).max() < 1e-14
        n_e += 2.0 * f.sum()
    assert abs(n_e - s["n_electrons"]) < 1e-9 * s["n_electrons"]
    assert sorted(set(int(x) for x in s["n_orb"])) == list(range(1, 17))


def test_ragged_and_maxdim_electron_count():
    for name in ("mixed27", "maxdim"):
        s = synth.small(name)
        r = oracle.density_build(s)
        assert abs(r["n_e"] - s["n_electrons"]) < 1e-9 * s["n_electrons"], name
        for i in range(0, s["n_atoms"], 7):
            for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
                if s["col"][b] == i:
                    m = s["n_orb"][i]
                    o = s["blk_off"][b]
                    d = r["D"][o: o + m * m].reshape(m, m)
                    assert np.abs(d - d.T).max() < 1e-12, name
    assert max(synth.small("mixed27")["n_orb"]) == 16
