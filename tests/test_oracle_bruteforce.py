"""Brute force in 40-digit arithmetic (mpmath) on a tiny system: the whole DC-LNO build,
LNOs with a complex-conjugate pair included, against the FP64 oracle.

The mpmath side is written from the paper independently of the oracle: its own distance
and region rule (Sec. III), Lambda (Eq. 17), general eigendecomposition (Eq. 20), kept
span (Eq. 22), cluster matrices (Eq. 26), Cholesky-reduced eigenproblem, weights, mu by
bisection and density rows (Eq. 24, 27)."""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

import oracle  # noqa: E402
from pair_systems import tiny_pair_system  # noqa: E402

mp.mp.dps = 40


def _tiny():
    return tiny_pair_system()


def _blk(s, vals, i, j):
    rp, col = s["row_ptr"], s["col"]
    for b in range(rp[i], rp[i + 1]):
        if col[b] == j:
            m1, m2 = s["n_orb"][i], s["n_orb"][j]
            return mp.matrix(vals[s["blk_off"][b]: s["blk_off"][b] + m1 * m2].reshape(m1, m2).tolist())
    return None


def _mp_regions(s):
    n = s["n_atoms"]
    L = s["cell"][0, 0]
    out = []
    for i in range(n):
        d = []
        for j in range(n):
            dx = (s["pos"][j, 0] - s["pos"][i, 0]) % L
            dx = min(dx, L - dx)
            d.append((round(dx, 9), j))
        c = sorted(x for x in d if x[0] <= s["r_L"] + 1e-9)
        fna = set(s["col"][s["row_ptr"][i]: s["row_ptr"][i + 1]].tolist())
        nf = len(fna)
        target = nf + s["kappa"] * (len(c) - nf)
        dists = sorted(set(x[0] for x in c))
        r_s = next(r for r in dists if sum(1 for x in c if x[0] <= r) >= target)
        short = [j for dd, j in c if dd <= r_s]
        long = [j for dd, j in c if dd > r_s]
        out.append((short, long))
    return out


def _mp_lno(s, dprev, j, k_fixed):
    m = s["n_orb"][j]
    lam = mp.zeros(m, m)
    for b in range(s["row_ptr"][j], s["row_ptr"][j + 1]):
        k = s["col"][b]
        lam += _blk(s, dprev, j, k) * _blk(s, s["S"], k, j)
    ev, er = mp.eig(lam)
    order = sorted(range(m), key=lambda t: (-mp.re(ev[t]), t))
    cols = []
    t = 0
    kept = 0
    pair = False
    while kept < k_fixed:
        v = er[:, order[t]]
        if abs(mp.im(ev[order[t]])) > mp.mpf(10) ** -30:
            cols.append([mp.re(x) for x in v])
            cols.append([mp.im(x) for x in v])
            kept += 2
            t += 2
            pair = True
        else:
            cols.append([mp.re(x) for x in v])
            kept += 1
            t += 1
    B = mp.matrix(cols).T
    Sjj = _blk(s, s["S"], j, j)
    G = B.T * Sjj * B
    e, u = mp.eigsy(G)
    Gm12 = u * mp.diag([1 / mp.sqrt(x) for x in e]) * u.T
    return B * Gm12, pair


def _mp_build(s, dprev, ranks):
    regions = _mp_regions(s)
    us = {}
    n_pairs = 0
    for j in range(s["n_atoms"]):
        us[j], pair = _mp_lno(s, dprev, j, int(ranks[j]))
        n_pairs += pair
    spectra, rows = [], []
    for i, (short, long) in enumerate(regions):
        members = short + long
        tr = [None] * len(short) + [us[j] for j in long]
        dims = [s["n_orb"][j] for j in short] + [us[j].cols for j in long]
        offs = np.concatenate([[0], np.cumsum(dims)]).astype(int)
        d = int(offs[-1])
        Hc, Sc = mp.zeros(d, d), mp.zeros(d, d)
        for a, ja in enumerate(members):
            for b, jb in enumerate(members):
                hb = _blk(s, s["H"], ja, jb)
                if hb is None:
                    continue
                sb = _blk(s, s["S"], ja, jb)
                if tr[a] is not None:
                    hb, sb = tr[a].T * hb, tr[a].T * sb
                if tr[b] is not None:
                    hb, sb = hb * tr[b], sb * tr[b]
                for p in range(hb.rows):
                    for q in range(hb.cols):
                        Hc[offs[a] + p, offs[b] + q] = hb[p, q]
                        Sc[offs[a] + p, offs[b] + q] = sb[p, q]
        Lc = mp.cholesky(Sc)
        Li = mp.inverse(Lc)
        A = Li * Hc * Li.T
        A = (A + A.T) / 2
        e, y = mp.eigsy(A)
        C = Li.T * y
        m0 = s["n_orb"][i]
        SC = Sc * C
        w = [sum(C[a, mu] * SC[a, mu] for a in range(m0)) for mu in range(d)]
        spectra.append(([e[t] for t in range(d)], w))
        fna = s["col"][s["row_ptr"][i]: s["row_ptr"][i + 1]].tolist()
        rws = {j: [[C[offs[members.index(j)] + p, mu] for mu in range(d)] for p in range(s["n_orb"][j])] for j in fna}
        rows.append(rws)
    kT, g = mp.mpf(s["kT"]), 2
    allp = [(e, w) for ev, ww in spectra for e, w in zip(ev, ww)]
    f = lambda x: 1 / (1 + mp.exp(x))  # noqa: E731
    lo = min(e for e, _ in allp) - 40 * kT
    hi = max(e for e, _ in allp) + 40 * kT
    for _ in range(140):
        mid = (lo + hi) / 2
        nmid = g * sum(f((e - mid) / kT) * w for e, w in allp)
        if nmid < s["n_electrons"]:
            lo = mid
        else:
            hi = mid
    mu = (lo + hi) / 2
    dvals = np.zeros_like(s["S"])
    for i in range(s["n_atoms"]):
        ev = spectra[i][0]
        occ = [f((e - mu) / kT) for e in ev]
        ci = rows[i][i]
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            cj = rows[i][j]
            blk = [[float(sum(ci[p][t] * occ[t] * cj[q][t] for t in range(len(ev)))) for q in range(len(cj))]
                   for p in range(len(ci))]
            dvals[s["blk_off"][b]: s["blk_off"][b] + len(ci) * len(cj)] = np.array(blk).ravel()
    return float(mu), dvals, n_pairs


def test_bruteforce_40_digits():
    s, dprev = _tiny()
    ref = oracle.density_build(s, dprev=dprev, fixed_rank=2, workers=1)
    ranks = ref["ranks"]
    mu, dvals, n_pairs = _mp_build(s, dprev, ranks)
    # the instance must exercise a kept complex-conjugate pair of Lambda
    assert n_pairs >= 1
    assert abs(mu - ref["mu"]) < 1e-12
    assert np.abs(dvals - ref["D"]).max() < 1e-12
