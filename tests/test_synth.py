"""Seeded input generator: determinism, symmetry, SPD overlap, distance-cutoff pattern."""
import numpy as np

import synth


def test_deterministic_and_symmetric():
    a = synth.small("sc27")
    b = synth.small("sc27")
    assert np.array_equal(a["H"], b["H"]) and np.array_equal(a["S"], b["S"])
    for key in ("H", "S"):
        m = synth.bsr_to_scipy(a, a[key]).toarray()
        assert np.abs(m - m.T).max() == 0.0


def test_overlap_spd_and_pattern():
    s = synth.small("fcc_slab")
    S = synth.bsr_to_scipy(s, s["S"]).toarray()
    assert np.linalg.eigvalsh(S)[0] >= 0.2
    # pattern = atoms within the third fcc shell (free z axis)
    pos, cell = s["pos"], s["cell"]
    for i in (0, 17, 100):
        d = pos - pos[i]
        for ax in range(3):
            if s["periodic"][ax]:
                d[:, ax] -= cell[ax, ax] * np.round(d[:, ax] / cell[ax, ax])
        r = np.sqrt((d * d).sum(1))
        expect = np.nonzero(r <= synth.SHELLS["fcc"][2] + 1e-6)[0]
        got = s["col"][s["row_ptr"][i]: s["row_ptr"][i + 1]]
        assert np.array_equal(np.sort(expect), got)


def test_config_sizes():
    s = synth.config(0)
    assert s["n_atoms"] == 64 and s["n_basis"] == 256 and s["n_electrons"] == 256.0
    assert np.all(np.diff(s["row_ptr"]) == 54)
