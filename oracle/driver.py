"""One DC-LNO density build, in the order of the paper's procedure (Sec. II.C, (i)-(v)).

(i)   LNOs of every atom from the previous density matrix (skipped for plain DC);
(ii)  cluster matrices with PAO/LNO blocks for every atom;
(iii) the cluster eigenproblems;
(iv)  one chemical potential for all clusters;
(v)   density rows of every atom.
Clusters are independent, so (ii)-(iii) and (v) run in a process pool, one cluster per
task, each worker on one BLAS thread.
"""
from __future__ import annotations

import os
import time
import multiprocessing as mp

import numpy as np

from .regions import plan_regions
from .lno import all_lnos
from .cluster import solve_cluster
from .density import (bisect_mu, density_rows, energy_density_rows, band_energy_and_count, window_rows,
                      window_weights)

_G = {}


def _init_worker():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass


def _solve(i):
    out = solve_cluster(_G["sys"], _G["regions"][i], _G["us"], _G["ranks"], keep_rows=_G["keep_rows"])
    if _G["mu"] is not None:
        mu, kT = _G["mu"], _G["kT"]
        if "rows" not in out:
            out = solve_cluster(_G["sys"], _G["regions"][i], _G["us"], _G["ranks"], keep_rows=True)
        ci = out["rows"][int(_G["regions"][i].center)]
        out["D"] = density_rows(ci, out["rows"], out["eps"], mu, kT)
        if _G.get("energy"):
            out["E"] = energy_density_rows(ci, out["rows"], out["eps"], mu, kT)
        if _G.get("window") is not None:
            out["W"] = window_rows(ci, out["rows"], out["eps"], *_G["window"])
        del out["rows"]
    return i, out


def _map(fn, items, workers):
    if workers <= 1 or len(items) <= 1:
        return [fn(i) for i in items]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init_worker) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (8 * workers)))


def _row_budget():
    """Bytes of coefficient rows a build may keep between its two passes: a quarter of the
    free host memory (at least 3 GB)."""
    try:
        import psutil
        return max(3e9, 0.25 * float(psutil.virtual_memory().available))
    except Exception:  # pragma: no cover
        return 3e9


def default_workers():
    return int(os.environ.get("LDC_ORACLE_WORKERS", min(16, os.cpu_count() or 1)))


def density_build(sysd, dprev=None, fixed_rank=None, mu=None, clusters=None, workers=None,
                  lno=None, regions=None, verbose=False, energy=False, window=None):
    """One density build.

    dprev: previous density matrix (BSR values) for the LNOs; None or lno=False gives plain
    DC.  fixed_rank: None, int, or per-atom array overriding the LNO rank rule.  mu: if
    given, no bisection; density rows at this chemical potential.  clusters: restrict to
    these atoms (needs mu for density rows).  Returns a dict with D (BSR values, rows of
    the computed clusters), mu, e_band, n_e, spectra {i: (eps, w)}, ranks, us, regions,
    dims, iters and timings.  energy: also the energy density rows (Eq. 25) as E and
    tr_es = g Tr(E S).  window: (e_lo, e_hi, kT) -- also the windowed density rows as W,
    tr_ws = g Tr(W S) and window_count = g sum_i sum_mu w(eps) w_mu (the projector of
    Sec. II.B with another energy window).
    """
    t0 = time.time()
    kT = sysd["kT"]
    g = float(sysd.get("spin_g", 2))
    if lno is None:
        lno = bool(sysd.get("lno", True)) and dprev is not None
    if regions is None:
        regions = plan_regions(sysd, lno=lno)
    us = ranks = None
    if lno:
        us, _, ranks = all_lnos(sysd, dprev, fixed_rank=fixed_rank)
    t_lno = time.time()
    n = sysd["n_atoms"]
    idx = list(range(n)) if clusters is None else [int(c) for c in clusters]
    workers = default_workers() if workers is None else workers
    # keep the coefficient rows in one pass when they fit comfortably in memory
    est = 0
    for i in idx[: min(len(idx), 8)]:
        r = regions[i]
        est += 8 * 9 * (r.n_fna + 1) * 9 * len(r.members)
    est = est / max(1, min(len(idx), 8)) * len(idx)
    keep_rows = est < _row_budget()
    _G.update(sys=sysd, regions=regions, us=us, ranks=ranks, keep_rows=keep_rows and mu is None,
              mu=mu, kT=kT, energy=energy, window=window)
    res = dict(_map(_solve, idx, workers))
    t_solve = time.time()
    spectra = {i: (res[i]["eps"], res[i]["w"]) for i in idx}
    iters = 0
    if mu is None:
        if clusters is not None:
            raise ValueError("a cluster subset needs an explicit chemical potential")
        mu, iters = bisect_mu([spectra[i] for i in idx], sysd["n_electrons"], kT, g)
        if keep_rows:
            for i in idx:
                r = res[i]
                res[i]["D"] = density_rows(r["rows"][i], r["rows"], r["eps"], mu, kT)
                if energy:
                    res[i]["E"] = energy_density_rows(r["rows"][i], r["rows"], r["eps"], mu, kT)
                if window is not None:
                    res[i]["W"] = window_rows(r["rows"][i], r["rows"], r["eps"], *window)
        else:
            _G.update(mu=mu)
            res2 = dict(_map(_solve, idx, workers))
            for i in idx:
                res[i]["D"] = res2[i]["D"]
                if energy:
                    res[i]["E"] = res2[i]["E"]
                if window is not None:
                    res[i]["W"] = res2[i]["W"]
    t_mu = time.time()
    row_ptr, col, blk_off, n_orb = sysd["row_ptr"], sysd["col"], sysd["blk_off"], sysd["n_orb"]

    def assemble(key):
        vals = np.zeros_like(sysd["S"])
        for i in idx:
            blk = res[i][key]
            for b in range(row_ptr[i], row_ptr[i + 1]):
                j = int(col[b])
                vals[blk_off[b]: blk_off[b] + n_orb[i] * n_orb[j]] = blk[j].ravel()
        return vals

    dvals = assemble("D")
    e_band, n_e = band_energy_and_count(sysd, dvals, g)
    e_spec = g * sum(float(np.sum(0.5 * (1 - np.tanh(0.5 * (spectra[i][0] - mu) / kT)) * spectra[i][0] * spectra[i][1]))
                     for i in idx)
    out = dict(D=dvals, mu=mu, e_band=e_band, n_e=n_e, e_band_spectral=e_spec, spectra=spectra,
               ranks=ranks, us=us, regions=regions, dims={i: res[i]["dim"] for i in idx}, iters=iters,
               times=dict(lno=t_lno - t0, solve=t_solve - t_lno, mu_rows=t_mu - t_solve, total=time.time() - t0))
    if energy:
        out["E"] = assemble("E")
        out["tr_es"] = g * float(np.dot(out["E"], sysd["S"]))
    if window is not None:
        out["W"] = assemble("W")
        out["tr_ws"] = g * float(np.dot(out["W"], sysd["S"]))
        out["window_count"] = g * sum(float(np.sum(window_weights(spectra[i][0], *window) * spectra[i][1]))
                                      for i in idx)
    if verbose:
        print(f"[oracle] {sysd.get('name')} clusters={len(idx)} mu={mu:.12f} e_band={e_band:.10f} "
              f"times={out['times']}", flush=True)
    return out
