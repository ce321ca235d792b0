"""Benchmark: atoms/s per DC-LNO density build on one MI355X.

One step = one whole density build of the hot path through the C ABI:
  ldc_lno     (Lambda, LNO eigensolve and selection, from the previous build's density),
  ldc_solve   (gather with LNO contraction, Cholesky, standard form, tridiagonalization,
               divide-and-conquer),
  ldc_density (chemical potential by bisection over all clusters, density rows).
Default workload: the metallic fcc slab (10x10x10 cells, periodic in x and y, 80 vacancies:
3920 atoms x 9 orbitals = 35280 basis functions, r_L = sqrt(5) d_NN, LNO rank =
clamp(#{lambda >= 1e-3}, 2, 6), kT = 0.01 Ha, half filling), FP64, synthetic seeded inputs.
Step 0 (untimed) is a plain-DC build whose density seeds the LNOs, as at the start of an
SCF cycle; every later step takes the previous step's density.

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (vector and matrix)
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E


def stage_work(dims):
    """Algorithmic FP64 flops of the matrix-core stages for clusters of dimension d, by the
    per-cluster LAPACK counts of the operation each stage performs: Cholesky d^3/3, standard
    form d^3, reduction to band form 4 d^3 / 3 (the whole tridiagonalization's count)."""
    d = dims.astype(np.float64)
    return {
        "potrf": float(np.sum(d ** 3 / 3.0)),
        "sygst": float(np.sum(d ** 3)),
        "sy2sb": float(np.sum(4.0 * d ** 3 / 3.0)),
    }


def executed_flops(dims, n_orb, b=32):
    """FP64 flops this design executes in the eigensolve (potrf .. stedc) per build: Cholesky
    d^3/3; standard form with the triangular inverse d^3/3, P = L^-1 H_L d^3/3 and
    A = P L^-T + L^-1 P^T 2 d^3/3; band reduction 4 d^3/3; bulge chasing 6 b d^2 (12 b^2 per
    step, d^2 / 2b steps); the 2M tracked columns through Q2 and the merges 8 M d^2.  No
    eigenvector matrix and no back-transform are formed (the O(d^3) part is 3 d^3)."""
    d = dims.astype(np.float64)
    m = np.asarray(n_orb, dtype=np.float64)
    return float(np.sum(3.0 * d ** 3 + 6.0 * b * d ** 2 + 8.0 * m * d ** 2))


def sb2st_min_bytes(dims, b=32):
    """HBM bytes the band-to-tridiagonal step cannot avoid: the lower band (b + 1 diagonals)
    read once, the bulge-chasing reflectors (n - 1 - s entries for sweep s) written once, the
    diagonal and off-diagonal written once."""
    total = 0.0
    for n in np.unique(dims):
        n = int(n)
        cnt = int(np.sum(dims == n))
        band = sum(min(b + 1, n - c) for c in range(n))
        refl = sum(n - 1 - s for s in range(0, max(0, n - 2)))
        total += cnt * 8.0 * (band + refl + 2 * n)
    return total


def sb2st_design_bytes(dims, b=32):
    """Bytes this design's chase moves through memory.  Sweeps go in pairs (s, s + 1), s even, on
    one wavefront: the first sweep's steps read their windows (the lower triangle of the len x len
    diagonal block and the nr x len block below it), the second sweep's steps write theirs (its
    windows are formed in registers from the first sweep's), and every step writes its reflector
    (len doubles).  The first sweep also writes the diagonal entry of column s + 1 (step 0), the
    first column's entries past the first R row (nr - 1, later steps) and, when the second sweep has
    one step fewer, its last window but the first column; the second sweep reads the first column
    of a window the first sweep does not reach (at most b + 1 doubles).  A lone last sweep reads
    and writes its windows.  Sweep s, step j: r0 = s + 1 + j b, len = min(b, d - r0),
    nr = min(b, d - r0 - len), steps while r0 <= d - 2.  Step 0's column s (32 doubles read, 32
    written) is left out."""
    def steps(n, s):
        return 0 if s > n - 3 else (n - 3 - s) // b + 1

    def window(n, s, j):
        r0 = s + 1 + j * b
        ln = min(b, n - r0)
        nr = max(0, min(b, n - r0 - ln))
        return ln, nr, ln * (ln + 1) // 2 + nr * ln

    total = 0.0
    for n in np.unique(dims):
        n = int(n)
        cnt = int(np.sum(dims == n))
        per = 0
        for s in range(0, n - 2, 2):
            J0, J1 = steps(n, s), steps(n, s + 1)
            if s + 1 > n - 3:
                for j in range(J0):
                    ln, nr, win = window(n, s, j)
                    per += 2 * win + ln
                continue
            for j in range(J0):
                ln, nr, win = window(n, s, j)
                per += win + ln
                if j == 0:
                    per += 1
                elif j == J0 - 1 and J1 <= j:
                    per += win - (ln + nr) + max(nr - 1, 0)
                else:
                    per += max(nr - 1, 0)
            for j in range(J1):
                ln, nr, win = window(n, s + 1, j)
                per += win + ln
                r0c = s + 1 + (j + 1) * b
                if j + 1 >= J0 and r0c <= n - 1:
                    per += min(b + 1, n - r0c)
        total += cnt * 8.0 * per
    return total


def copy_probe(mib):
    """Three plain device-to-device copies of a known size: the per-dispatch FETCH_SIZE and
    WRITE_SIZE they read give the factor that turns those counters into HBM bytes."""
    import torch
    n = mib * 2 ** 20 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}), flush=True)


def kernel_source_hash(source):
    """Hash of a kernel's HIP source file and the local headers it includes (ties stored counters
    to the code they were taken on)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1809_05637_amd", "csrc")
    seen, todo = [], [source]
    while todo:
        name = todo.pop()
        if name in seen or not os.path.exists(os.path.join(csrc, name)):
            continue
        seen.append(name)
        with open(os.path.join(csrc, name)) as f:
            todo += re.findall(r'^#include "([^"]+)"', f.read(), re.M)
    h = hashlib.sha256()
    for name in sorted(seen):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


# kernel -> source file (the dominant kernels whose counters can be stored)
KERNEL_SOURCE = {"sb2st_kernel": "k_tridiag.hip", "sy2sb_kernel": "k_tridiag.hip",
                 "sygst_kernel": "k_solve.hip", "potrf_kernel": "k_solve.hip", "stedc_kernel": "k_dc.hip"}


def stored_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary (lines
    `hbm_bytes_per_launch: X` and `source_hash: H`), or None when the summary is missing or was
    taken on other kernel sources."""
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCE:
        return None
    with open(path) as f:
        text = f.read()
    h = re.search(r"^source_hash:\s*(\S+)", text, re.M)
    b = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not h or not b or h.group(1) != kernel_source_hash(KERNEL_SOURCE[kernel]):
        return None
    return float(b.group(1))


def host_workers():
    """Oracle pool size: the host cores this process may run on, at most 16 (the host share
    that goes with one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(s, sample_n, seed=0):
    """The CPU oracle on a sample of clusters of the same workload (test infrastructure): the
    SCF benchmark's baseline (one build's cost, extrapolated from the sample)."""
    import oracle
    t_start = time.time()
    rng = np.random.default_rng(seed)
    clusters = np.sort(rng.choice(s["n_atoms"], size=min(sample_n, s["n_atoms"]), replace=False))
    # previous density for the LNOs: the half-filled atomic limit (0.5 S_ii^{-1} on the diagonal
    # blocks).  The oracle's cost does not depend on these values.
    dprev = np.zeros_like(s["S"])
    rp, col, off, no = s["row_ptr"], s["col"], s["blk_off"], s["n_orb"]
    for i in range(s["n_atoms"]):
        for b in range(rp[i], rp[i + 1]):
            if col[b] == i:
                m = no[i]
                sii = s["S"][off[b]: off[b] + m * m].reshape(m, m)
                dprev[off[b]: off[b] + m * m] = (0.5 * np.linalg.inv(sii)).ravel()
    workers = host_workers()
    r = oracle.density_build(s, dprev=dprev, mu=0.0, clusters=clusters, workers=workers)
    t = r["times"]
    per_cluster = t["solve"] / len(clusters)
    est = t["lno"] + per_cluster * s["n_atoms"] + t["mu_rows"] * s["n_atoms"] / len(clusters)
    return {"value": s["n_atoms"] / est, "unit": "atoms/s", "cores": workers, "kind": "oracle",
            "sample": (f"{len(clusters)} of {s['n_atoms']} clusters of the same DC-LNO build (LNOs of all atoms, "
                       f"cluster eigensolves and density rows at a fixed mu) in a {workers}-process pool; "
                       f"{time.time() - t_start:.1f} s wall; build time extrapolated to all clusters: {est:.1f} s")}


def oracle_builds(s, log):
    """The oracle's own chain on the benchmark input (test infrastructure, the cpu_baseline
    leg): its plain-DC build (untimed), then the DC-LNO build from that density, timed whole
    (all clusters, bisection over all of them, every density row; no sampling)."""
    import oracle
    workers = host_workers()
    t0 = time.time()
    r0 = oracle.density_build(s, dprev=None, workers=workers)
    t1 = time.time()
    log(f"[bench] oracle plain-DC build: {t1 - t0:.1f} s on {workers} processes")
    r1 = oracle.density_build(s, dprev=r0["D"], workers=workers)
    t2 = time.time()
    log(f"[bench] oracle DC-LNO build: {t2 - t1:.1f} s  mu={r1['mu']:.12f}  "
        f"E_band/atom={r1['e_band'] / s['n_atoms']:.12f}")
    base = {"value": round(s["n_atoms"] / (t2 - t1), 3), "unit": "atoms/s", "cores": workers, "kind": "oracle",
            "sample": (f"the whole DC-LNO build of the same input ({s['n_atoms']} clusters: LNOs of every atom from "
                       f"the oracle's own plain-DC density, every cluster eigensolve, the bisection over all of "
                       f"them and every density row) in a {workers}-process pool: {t2 - t1:.1f} s wall; its "
                       f"plain-DC build that seeds the LNOs took {t1 - t0:.1f} s and is not counted")}
    return base, r0, r1


def accuracy_vs_oracle(s, ref, D, mu, eb, ne, ranks):
    """The timed build against the oracle's build of the same input (Eq. 13, 24 with 27):
    band energy per atom, density rows element by element, chemical potential, electron
    count (g Tr(D S) from the returned rows against N_e, and against the oracle's), ranks."""
    n = s["n_atoms"]
    return {"vs": "oracle DC-LNO build of the same input (its own plain-DC density for the LNOs)",
            "dE_band_per_atom": abs(eb - ref["e_band"]) / n,
            "max_dD": float(np.max(np.abs(D - ref["D"]))),
            "dmu": abs(mu - ref["mu"]),
            "dN_e_strict": abs(ne - s["n_electrons"]),
            "dN_e_vs_oracle": abs(ne - ref["n_e"]),
            "ranks_equal": bool(np.array_equal(np.asarray(ranks), np.asarray(ref["ranks"]))),
            "e_band_per_atom": eb / n, "mu": mu}


def scf_bench(s, plan, H0, S, rule, use_lno, args, log):
    """Toy SCF loop: one untimed step (plain DC, seeds the LNOs), then args.scf steps timed with
    HIP events on the plan's stream; then Mulliken, potential and mixing timed alone."""
    import torch
    import paper_1809_05637_amd.scf as scf
    stream = torch.cuda.current_stream()
    U, alpha = args.scf_u, args.scf_alpha
    ev = []

    def on_step(k, rec):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        ev.append(e)
        log(f"[scf] step {k}: residual {rec['residual']:.3e} mu={rec['mu']:.10f} "
            f"E_band/atom={rec['e_band'] / s['n_atoms']:.10f}")
        if k == 0:
            plan.profile(True)

    torch.cuda.synchronize()
    hist = scf.scf_loop(plan, H0, S, s["n_electrons"], s["kT"], U, alpha, args.scf + 1, lno=use_lno,
                        on_step=on_step, **rule)
    torch.cuda.synchronize()
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(len(ev) - 1)]
    ms_step = float(np.mean(ms))
    stages, builds = plan.stage_times()
    per_stage = {k: v / max(1, builds) for k, v in stages.items()}
    # the SCF kernels alone (10 calls each, on the last step's buffers)
    q0 = torch.empty(s["n_atoms"], dtype=torch.float64, device=S.device)
    plan.reference_populations(s["n_electrons"], q0)
    q_in, q_out, v = q0.clone(), torch.zeros_like(q0), torch.zeros_like(q0)
    D, H = torch.zeros_like(S), torch.empty_like(H0)

    def timed(fn, reps=10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_mull = timed(lambda: plan.mulliken(D, S, q_out))
    ms_pot = timed(lambda: plan.potential(H0, S, v, H))
    ms_mix = timed(lambda: plan.scf_mix(q_out, q_in, q0, U, alpha, v, want_residual=False))
    nb = float(len(s["S"])) * 8.0
    kern = {"mulliken_ms": round(ms_mull, 4), "potential_ms": round(ms_pot, 4), "mix_ms": round(ms_mix, 4),
            "mulliken_bytes": 2 * nb, "potential_bytes": 3 * nb,
            "mulliken_GBps": round(2 * nb / (ms_mull * 1e-3) / 1e9, 1),
            "potential_GBps": round(3 * nb / (ms_pot * 1e-3) / 1e9, 1), "hbm_peak_GBps": HBM_PEAK_GBS}
    log(f"[scf] {args.scf} timed steps: {ms_step:.1f} ms/step; kernels: " +
        ", ".join(f"{k}={v}" for k, v in kern.items()))
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("[scf] cpu baseline (oracle) ...")
        cb = cpu_baseline(s, args.cpu_sample)
        t0 = time.time()
        q = oracle.mulliken(s, s["S"])
        oracle.potential(s, s["H"], 0.1 * (q - oracle.reference_populations(s)))
        t_scf = time.time() - t0
        build_s = s["n_atoms"] / cb["value"]
        cpu = {"value": round(s["n_atoms"] / (build_s + t_scf), 3), "unit": "atoms/s", "cores": cb["cores"],
               "kind": "oracle",
               "sample": cb["sample"] + f"; plus the oracle's Mulliken populations and potential on the whole "
                                        f"system, one process: {t_scf:.2f} s"}
    out = {
        "metric": "atoms/s per toy SCF step (FP64 form; LNOs regenerated every step)",
        "value": round(s["n_atoms"] / (ms_step * 1e-3), 2),
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.scf,
        "warmup": 1,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": s["name"] + "_scf_fp64", "U": U, "alpha": alpha, "atoms": int(s["n_atoms"])},
        "residuals": [round(h["residual"], 8) for h in hist],
        "build_stage_ms": {k: round(v, 3) for k, v in per_stage.items()},
        "scf_kernels": kern,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    return out


def exact_band_energy(s):
    """Conventional O(N^3) reference of the sweep: all generalized eigenvalues of the whole
    system's Gamma-folded H and S (scipy), mu by bisection on g sum f = N_e, E_band = g sum f eps."""
    import scipy.linalg
    n_orb = np.asarray(s["n_orb"])
    offs = np.concatenate([[0], np.cumsum(n_orb)])
    hd = np.zeros((offs[-1], offs[-1]))
    sd = np.zeros_like(hd)
    for i in range(s["n_atoms"]):
        for b in range(s["row_ptr"][i], s["row_ptr"][i + 1]):
            j = s["col"][b]
            o, m = s["blk_off"][b], n_orb[i] * n_orb[j]
            hd[offs[i]:offs[i + 1], offs[j]:offs[j + 1]] = s["H"][o:o + m].reshape(n_orb[i], n_orb[j])
            sd[offs[i]:offs[i + 1], offs[j]:offs[j + 1]] = s["S"][o:o + m].reshape(n_orb[i], n_orb[j])
    e = scipy.linalg.eigh(hd, sd, eigvals_only=True)
    kT, g = s["kT"], 2.0
    f = lambda x: 0.5 * (1.0 - np.tanh(0.5 * x))  # noqa: E731
    lo, hi = e[0] - 40 * kT, e[-1] + 40 * kT
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if hi - lo <= 4e-16 * max(1.0, abs(mid)):
            break
        if g * np.sum(f((e - mid) / kT)) < s["n_electrons"]:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    return float(g * np.sum(f((e - mu) / kT) * e)), mu


def eq28_ratio(n_short, n_long, m_p, m_l):
    """Eq. 28 with the short and long atom counts of the cluster:
    t_DC-LNO / t_DC = [M_P n_short + M_L n_long]^3 / [M_P (n_short + n_long)]^3.  The paper's worked
    example (275 short, 190 long, 13 PAOs, 4 LNOs -> 0.37) evaluates it this way."""
    return (m_p * n_short + m_l * n_long) ** 3 / (m_p * (n_short + n_long)) ** 3


def eq28_kappa(n_f, n_s, m_p, m_l, kappa=0.3):
    """Eq. 28 as printed, with the buffer at exactly kappa N_S:
    [M_P (N_F + kappa N_S) + M_L (1 - kappa) N_S]^3 / [M_P (N_F + N_S)]^3."""
    return eq28_ratio(n_f + kappa * n_s, (1 - kappa) * n_s, m_p, m_l)


def _timed_build(plan, H, S, s, dprev, rule, D, stream):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ranks = plan.lno(S, dprev, want_ranks=dprev is not None, **rule)
    a.record(stream)
    plan.solve(H, S)
    mu, eb, ne = plan.density(s["n_electrons"], s["kT"], D)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b), mu, eb, ranks


def sweep_bench():
    """Error of plain DC and DC-LNO against exact diagonalization versus the cluster radius
    (Sec. IV, Fig. 5's measurement on synthetic systems), and t_DC-LNO / t_DC (solve + density,
    HIP events) against Eq. 28 and against the cube ratio of the actual dimensions."""
    import torch
    import synth
    import paper_1809_05637_amd as ldc
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {"metric": "band-energy error vs cluster radius and DC-LNO/DC time ratio", "unit": "Ha/atom",
           "n_gpus": 1, "dtype": "f64", "data": "synthetic", "systems": {}}
    for name, shells in (("dia216", synth.SHELLS["diamond"][1:8]), ("fcc256", synth.SHELLS["fcc"][2:6])):
        s = synth.small(name)
        e_ex, mu_ex = exact_band_energy(s)
        n = s["n_atoms"]
        log(f"[sweep] {name}: {n} atoms, exact E_band/atom {e_ex / n:.12f}")
        H = torch.from_numpy(s["H"]).to(dev)
        S = torch.from_numpy(s["S"]).to(dev)
        D0, D1 = torch.zeros_like(S), torch.zeros_like(S)
        rule = dict(lambda_th=s["lambda_th"], k_min=s["k_min"], k_max=s["k_max"],
                    fixed_rank=s["fixed_k"] if s["fixed_k"] >= 0 else None)
        pts = []
        for r in shells:
            r_L = r * (1 + 1e-9)
            plan = ldc.Plan(s["pos"], s["cell"], s["periodic"], s["n_orb"], s["row_ptr"], s["col"], r_L,
                            kappa=s["kappa"], stream=stream)
            ptr, _, lng = ldc.regions(s["pos"], s["cell"], s["periodic"], s["n_orb"], s["row_ptr"], s["col"], r_L)
            n_mem = np.diff(ptr)
            n_long = np.add.reduceat(lng, ptr[:-1]) if len(lng) else np.zeros(n, dtype=int)
            n_f = np.diff(s["row_ptr"])
            t_dc, _, e_dc, _ = _timed_build(plan, H, S, s, None, rule, D0, stream)
            dims_dc = plan.cluster_dims()
            pt = {"r_L": round(r, 4), "atoms": float(n_mem.mean()), "long": float(n_long.mean()),
                  "dim_dc": int(dims_dc.max()), "err_dc": abs(e_dc - e_ex) / n, "ms_dc": round(t_dc, 3)}
            if n_long.max() > 0:
                t_l, _, e_l, ranks = _timed_build(plan, H, S, s, D0, rule, D1, stream)
                dims_l = plan.cluster_dims()
                m_l = float(np.mean(ranks))
                pt.update(dim_lno=int(dims_l.max()), err_lno=abs(e_l - e_ex) / n, ms_lno=round(t_l, 3),
                          mean_rank=m_l, cube_ratio=float(np.sum(dims_l.astype(float) ** 3) / np.sum(dims_dc.astype(float) ** 3)),
                          eq28=float(np.mean(eq28_ratio(n_mem - n_long, n_long, float(s["n_orb"][0]), m_l))),
                          eq28_kappa=float(np.mean(eq28_kappa(n_f, n_mem - n_f, float(s["n_orb"][0]), m_l))))
            plan.close()
            pts.append(pt)
            log(f"[sweep] {name} r_L={r:.3f}: " + ", ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                                                          for k, v in pt.items()))
        out["systems"][name] = {"atoms": n, "basis": int(s["n_basis"]), "kT": s["kT"], "exact_e_band_per_atom": e_ex / n,
                                "points": pts}
    # the benchmark workload: plain DC (PAOs everywhere) against DC-LNO, two builds each
    s = synth.load_config(2)
    H = torch.from_numpy(s["H"]).to(dev)
    S = torch.from_numpy(s["S"]).to(dev)
    D0, D1 = torch.zeros_like(S), torch.zeros_like(S)
    rule = dict(lambda_th=s["lambda_th"], k_min=s["k_min"], k_max=s["k_max"],
                fixed_rank=s["fixed_k"] if s["fixed_k"] >= 0 else None)
    plan = ldc.Plan.from_system(s, stream=stream)
    ptr, _, lng = ldc.regions(s["pos"], s["cell"], s["periodic"], s["n_orb"], s["row_ptr"], s["col"], s["r_L"])
    n_mem = np.diff(ptr)
    n_long = np.add.reduceat(lng, ptr[:-1])
    n_f = np.diff(s["row_ptr"])
    t_dc = [_timed_build(plan, H, S, s, None, rule, D0, stream)[0] for _ in range(2)]
    dims_dc = plan.cluster_dims()
    res = [_timed_build(plan, H, S, s, D0, rule, D1, stream) for _ in range(2)]
    dims_l = plan.cluster_dims()
    m_l = float(np.mean(res[-1][3]))
    t_l = [r[0] for r in res]
    plan.close()
    out["workload"] = {
        "name": s["name"], "atoms": int(s["n_atoms"]), "ms_dc": round(min(t_dc), 3), "ms_lno": round(min(t_l), 3),
        "measured_ratio": round(min(t_l) / min(t_dc), 4),
        "cube_ratio": round(float(np.sum(dims_l.astype(float) ** 3) / np.sum(dims_dc.astype(float) ** 3)), 4),
        "eq28_mean": round(float(np.mean(eq28_ratio(n_mem - n_long, n_long, 9.0, m_l))), 4),
        "eq28_kappa_mean": round(float(np.mean(eq28_kappa(n_f, n_mem - n_f, 9.0, m_l))), 4), "mean_rank": round(m_l, 3),
        "dim_dc_mean": round(float(dims_dc.mean()), 1), "dim_lno_mean": round(float(dims_l.mean()), 1)}
    log(f"[sweep] workload: {out['workload']}")
    return out


def window_bench(s, plan, H, S, rule, log, half_width=0.5, k_window=4):
    """Energy-window LNOs (Sec. II.B): after a plain-DC build and a DC-LNO build, the windowed
    density rows over mu +- half_width (edge width kT), LNOs from them (k_window per atom), and a
    build with those LNOs; HIP events on the plan's stream, three repetitions, the minimum."""
    import torch
    stream = torch.cuda.current_stream()
    D0, D1, W = torch.zeros_like(S), torch.zeros_like(S), torch.zeros_like(S)
    plan.lno(S, None)
    plan.solve(H, S)
    plan.density(s["n_electrons"], s["kT"], D0)
    plan.lno(S, D0, want_ranks=False, **rule)
    plan.solve(H, S)
    mu, _, _ = plan.density(s["n_electrons"], s["kT"], D1)
    win = (mu - half_width, mu + half_width, s["kT"])

    def timed(fn, reps=3):
        best, res = None, None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = fn()
            b.record(stream)
            torch.cuda.synchronize()
            t = a.elapsed_time(b)
            best = t if best is None else min(best, t)
        return best, res

    ms_w, count = timed(lambda: plan.window_density(*win, W))
    ms_lno, ranks = timed(lambda: plan.lno(S, W, lambda_th=0.0, k_min=k_window, k_max=k_window))
    ms_build, (mu_w, eb_w, _) = timed(lambda: (plan.solve(H, S), plan.density(s["n_electrons"], s["kT"], D0))[1])
    log(f"[window] rows {ms_w:.2f} ms (count {count:.3f}), LNOs {ms_lno:.2f} ms, build {ms_build:.2f} ms")
    return {
        "metric": "energy-window LNOs: window rows, LNOs and build times (FP64 form)",
        "value": round(s["n_atoms"] / (ms_w * 1e-3), 2), "unit": "atoms/s (window rows)", "n_gpus": 1,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": s["name"] + "_window_fp64", "window_ha": [round(win[0], 6), round(win[1], 6)],
                   "kT": s["kT"], "lnos_per_atom": k_window},
        "ms_window_rows": round(ms_w, 3), "window_state_count": count, "ms_lno_from_window": round(ms_lno, 3),
        "ms_build_with_window_lnos": round(ms_build, 3), "e_band_per_atom": eb_w / s["n_atoms"],
        "density_rows_ms_note": "window rows run the density kernel with window weights (same cost as density rows)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="batched form without running the tuner")
    ap.add_argument("--no-mixed", action="store_true", help="skip the precision form (mixed FP32)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1809_05637_amd", "tune", "mi355x.json"),
                    help="tuning cache of the batched form (read, and written by the tuner when it has no entry)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--scf", type=int, default=0, metavar="K",
                    help="instead of the build benchmark: K timed steps of the toy SCF loop (LNOs regenerated "
                         "every step) after one untimed step, and the SCF kernels timed alone")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the build benchmark: band-energy error of plain DC and DC-LNO against "
                         "exact diagonalization versus the cluster radius (a gapped and a metallic system), "
                         "and the DC-LNO / DC time ratio on the benchmark workload against Eq. 28")
    ap.add_argument("--window", action="store_true",
                    help="instead of the build benchmark: energy-window density rows (mu +- 0.5 Ha) after a "
                         "DC-LNO build, LNOs from them and a build with those LNOs, timed")
    ap.add_argument("--scf-u", type=float, default=0.2)
    ap.add_argument("--scf-alpha", type=float, default=0.3)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    if args.sweep:
        print(json.dumps(sweep_bench()), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark times one density-matrix build on one GPU; --gpus must be 1 "
                                   "(the cluster loop would shard by atoms across GPUs, see the design notes)"}))
        sys.exit(2)
    import torch
    import synth
    import paper_1809_05637_amd as ldc

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    t0 = time.time()
    s = synth.load_config(args.config)
    log(f"[bench] config {args.config} {s['name']}: {s['n_atoms']} atoms, {s['n_basis']} basis, "
        f"{len(s['col'])} blocks ({time.time() - t0:.1f} s)")
    dev = torch.device("cuda:0")
    # a stream of its own (default priority): the batched form captures its builds there
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    H = torch.from_numpy(s["H"]).to(dev)
    S = torch.from_numpy(s["S"]).to(dev)
    torch.cuda.synchronize()
    t1 = time.time()
    plan = ldc.Plan.from_system(s, stream=stream)
    info = plan.info()
    log(f"[bench] plan: {time.time() - t1:.2f} s, max members {info['max_members']}, max PAO dim "
        f"{info['max_dim_pao']}, device memory {info['device_bytes'] / 2**30:.2f} GiB")
    rule = dict(lambda_th=s["lambda_th"], k_min=s["k_min"], k_max=s["k_max"],
                fixed_rank=s["fixed_k"] if s["fixed_k"] >= 0 else None)
    use_lno = bool(s["lno"])
    if args.window:
        print(json.dumps(window_bench(s, plan, H, S, rule, log)), flush=True)
        plan.close()
        return
    if args.scf > 0:
        print(json.dumps(scf_bench(s, plan, H, S, rule, use_lno, args, log)), flush=True)
        plan.close()
        return
    out = build_bench(s, args, log, H, S, plan, stream, rule, use_lno)
    print(json.dumps(out), flush=True)


def build_bench(s, args, log, H, S, plan, stream, rule, use_lno):
    """The FP64 forms on the benchmark workload.  Step 0 (untimed) is plain DC; its density D0
    is the previous density of every timed build, so that every timed build does the same work.
    Eager form: ldc_lno + ldc_solve + ldc_density per step with per-stage HIP events.  Batched
    form: one ldc_build per step, replayed from a HIP graph, size buckets and launch grids from
    the tuning cache (ldc_tune fills it when it has no entry for this device and workload)."""
    import torch
    import paper_1809_05637_amd as ldc
    Da, Db, Dc = torch.zeros_like(S), torch.zeros_like(S), torch.zeros_like(S)
    t2 = time.time()
    plan.lno(S, None)
    plan.solve(H, S)
    mu0, eb0, ne0 = plan.density(s["n_electrons"], s["kT"], Da)
    log(f"[bench] plain-DC build: {time.time() - t2:.2f} s  mu={mu0:.10f}  E_band/atom={eb0 / s['n_atoms']:.10f}")
    D0 = Da if use_lno else None
    ranks = plan.lno(S, D0, want_ranks=True, **rule)

    def step():
        plan.lno(S, D0, want_ranks=False, **rule)
        plan.solve(H, S)
        return plan.density(s["n_electrons"], s["kT"], Db)

    for w in range(args.warmup):
        tw = time.time()
        mu, eb, ne = step()
        log(f"[bench] eager warmup {w}: {time.time() - tw:.3f} s  mu={mu:.10f}")
    plan.profile(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for k in range(args.steps):
        mu, eb, ne = step()
        log(f"[bench] eager step {k}: mu={mu:.12f} E_band/atom={eb / s['n_atoms']:.12f} N_e(D)={ne:.9f}")
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_eager = ev0.elapsed_time(ev1) / args.steps
    stages, builds = plan.stage_times()
    dims = plan.cluster_dims()
    plan.profile(False)
    per_stage = {k: v / max(1, builds) for k, v in stages.items()}
    log("[bench] stage ms/build: " + ", ".join(f"{k}={v:.2f}" for k, v in per_stage.items()))
    log(f"[bench] dims: min {dims.min()} mean {dims.mean():.1f} max {dims.max()}; eager {ms_eager:.1f} ms/build")
    D_eager = Db.cpu().numpy()

    # batched form: tuned buckets, one graph-replayed ldc_build per step
    cache = args.tune_cache
    bplan = ldc.Plan.from_system(s, stream=stream, batched=True, use_graph=True, tune_cache=cache)
    bplan.build(H, S, None, s["n_electrons"], s["kT"], Dc)
    bplan.build(H, S, D0, s["n_electrons"], s["kT"], Dc, **rule)
    tune_ms = None
    if bplan.info()["tuned"] != 2 and not args.no_tune:
        tt = time.time()
        tune_ms = bplan.tune(H, S, D0, s["n_electrons"], s["kT"], Dc, **rule)
        log(f"[bench] tuned in {time.time() - tt:.1f} s: {tune_ms:.1f} ms/build, cache {cache}")
    for w in range(max(1, args.warmup)):
        bplan.build(H, S, D0, s["n_electrons"], s["kT"], Dc, **rule)
    torch.cuda.synchronize()
    ev0.record(stream)
    for k in range(args.steps):
        mu_b, eb_b, ne_b = bplan.build(H, S, D0, s["n_electrons"], s["kT"], Dc, **rule)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    binfo = bplan.info()
    buckets = bplan.buckets()
    bplan.close()
    D_gpu = Dc.cpu().numpy()
    log(f"[bench] batched form: {ms_step:.1f} ms/build ({len(buckets)} buckets, launch choices "
        f"{['default', 'tuned', 'cache'][binfo['tuned']]}, graph captures {binfo['graph_captures']}, "
        f"replays {binfo['graph_replays']}); max |D_batched - D_eager| = {np.abs(D_gpu - D_eager).max():.3e}")

    # precision form on the same input and the same previous density
    mixed = None
    if not args.no_mixed:
        mplan = ldc.Plan.from_system(s, stream=stream, batched=True, use_graph=True, tune_cache=cache,
                                     prec="mixed_fp32")
        Dm = torch.zeros_like(S)
        mplan.build(H, S, D0, s["n_electrons"], s["kT"], Dm, **rule)
        if mplan.info()["tuned"] != 2 and not args.no_tune:
            tt = time.time()
            mt = mplan.tune(H, S, D0, s["n_electrons"], s["kT"], Dm, **rule)
            log(f"[bench] mixed form tuned in {time.time() - tt:.1f} s: {mt:.1f} ms/build")
        for w in range(max(1, args.warmup)):
            mplan.build(H, S, D0, s["n_electrons"], s["kT"], Dm, **rule)
        torch.cuda.synchronize()
        ev0.record(stream)
        for k in range(args.steps):
            mu_m, eb_m, ne_m = mplan.build(H, S, D0, s["n_electrons"], s["kT"], Dm, **rule)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_m = ev0.elapsed_time(ev1) / args.steps
        ranks_m = mplan.lno(S, D0, want_ranks=True, **rule)
        mplan.solve(H, S)
        mplan.density(s["n_electrons"], s["kT"], Dm)
        resid = bisection_residual(mplan, s, mu_m)
        minfo = mplan.info()
        mplan.close()
        mixed = {"atoms_per_s": round(s["n_atoms"] / (ms_m * 1e-3), 2), "ms_per_build": round(ms_m, 3),
                 "speedup_vs_fp64_batched": round(ms_step / ms_m, 4),
                 "lowered": "H half of the gather and of the LNO contraction (FP32 values, FP32 arithmetic); "
                            "standard-form products P = L^-1 H_L and A = P L^-T + L^-1 P^T on FP32 matrix cores "
                            "with FP32 accumulation",
                 "fp64": "S gather and contraction, Cholesky and inverse of L, band reduction, bulge chasing, "
                         "divide-and-conquer, mu bisection, density rows",
                 "launch_choices": ["default", "tuned", "cache"][minfo["tuned"]],
                 "D": Dm.cpu().numpy(), "mu": mu_m, "e_band": eb_m, "n_e": ne_m, "ranks": ranks_m,
                 "bisection_residual": resid}
        log(f"[bench] mixed form: {ms_m:.1f} ms/build ({ms_step / ms_m:.3f}x the FP64 batched form); "
            f"max |D_mixed - D_fp64| = {np.abs(mixed['D'] - D_gpu).max():.3e}; bisection residual {resid:.3e}")

    work = stage_work(dims)
    dom = max(per_stage, key=per_stage.get)
    kern = dom + "_kernel"
    if dom == "sb2st":
        alg = sb2st_min_bytes(dims)
        achieved = alg / (per_stage[dom] * 1e-3) / 1e9
        roof = {"kernel": kern, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": stored_traffic(kern, s["name"]),
                "ms_per_launch": round(per_stage[dom], 3), "algorithmic_bytes": alg,
                "algorithmic": "lower band read once + reflectors, diagonal and off-diagonal written once",
                "design_traffic": sb2st_design_bytes(dims),
                "design_traffic_note": "sweeps in pairs on one wavefront: the first sweep's windows read, the "
                                       "second's written, reflectors written (this design's chase)"}
    elif dom in work:
        achieved = work[dom] / (per_stage[dom] * 1e-3) / 1e12
        roof = {"kernel": kern, "bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": stored_traffic(kern, s["name"]), "ms_per_launch": round(per_stage[dom], 3),
                "algorithmic_flops": work[dom]}
    else:
        roof = {"kernel": kern, "bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": None, "traffic": None, "ms_per_launch": round(per_stage[dom], 3)}
    roof["measured"] = "HIP events around the kernel on the plan's stream, eager builds of the same work"
    # the bulge chase against HBM whichever stage dominates: the method's minimum bytes and this
    # design's window traffic, per launch
    chase = None
    if per_stage.get("sb2st", 0.0) > 0:
        cmin, cdes = sb2st_min_bytes(dims), sb2st_design_bytes(dims)
        chase = {"kernel": "sb2st_kernel", "ms_per_launch": round(per_stage["sb2st"], 3), "min_bytes": cmin,
                 "min_gbs": round(cmin / (per_stage["sb2st"] * 1e-3) / 1e9, 2), "design_bytes": cdes,
                 "design_gbs": round(cdes / (per_stage["sb2st"] * 1e-3) / 1e9, 2),
                 "traffic": stored_traffic("sb2st_kernel", s["name"])}
    # the eigensolve as a whole (Cholesky .. divide-and-conquer) against the FP64 peak: executed
    # flops, and the tridiagonalization (band reduction + chase) against its LAPACK count
    eig_ms = sum(per_stage.get(k, 0.0) for k in ("potrf", "sygst", "sy2sb", "sb2st", "q2x", "stedc"))
    ex = executed_flops(dims, np.asarray(s["n_orb"]))
    tri_ms = per_stage.get("sy2sb", 0.0) + per_stage.get("sb2st", 0.0)
    tri_fl = float(np.sum(4.0 * dims.astype(np.float64) ** 3 / 3.0))
    eig = {"executed_flops": ex, "ms": round(eig_ms, 3),
           "tflops": round(ex / (eig_ms * 1e-3) / 1e12, 3) if eig_ms > 0 else None,
           "frac_fp64_peak": round(ex / (eig_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4) if eig_ms > 0 else None,
           "tridiagonalization": {"flops_4d3_3": tri_fl, "ms": round(tri_ms, 3),
                                  "frac_fp64_peak": round(tri_fl / (tri_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)
                                  if tri_ms > 0 else None},
           "lapack_equivalent_flops_7d3": float(np.sum(7.0 * dims.astype(np.float64) ** 3))}
    value = s["n_atoms"] / (ms_step * 1e-3)
    out = {
        "metric": "atoms/s per density-matrix build (FP64 form; the mixed FP32 form under forms)",
        "value": round(value, 2),
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": s["name"] + "_dclno_fp64", "atoms": int(s["n_atoms"]), "basis": int(s["n_basis"]),
                   "clusters": int(s["n_atoms"]), "dim_min": int(dims.min()), "dim_mean": round(float(dims.mean()), 1),
                   "dim_max": int(dims.max()), "kT": s["kT"], "form": "fp64 batched (hipGraph replay, tuned buckets)",
                   "lno_source": "plain-DC density of the same input (fixed for every timed build)"},
        "clusters_per_s": round(value, 2),
        "forms": {
            "fp64_batched": {"atoms_per_s": round(value, 2), "ms_per_build": round(ms_step, 3),
                             "buckets": buckets, "launch_choices": ["default", "tuned", "cache"][binfo["tuned"]],
                             "tune_ms": tune_ms, "graph_captures": binfo["graph_captures"],
                             "graph_replays": binfo["graph_replays"]},
            "fp64_eager": {"atoms_per_s": round(s["n_atoms"] / (ms_eager * 1e-3), 2),
                           "ms_per_build": round(ms_eager, 3),
                           "max_abs_diff_vs_batched": float(np.abs(D_gpu - D_eager).max())},
        },
        "stage_ms": {k: round(v, 3) for k, v in per_stage.items()},
        "roofline": roof,
        "bulge_chase": chase,
        "eigensolve": eig,
        "accuracy": {"n_e_from_D": ne_b, "n_electrons": s["n_electrons"], "mu": mu_b,
                     "e_band_per_atom": eb_b / s["n_atoms"]},
    }
    plan.close()
    if mixed is not None:
        out["forms"]["mixed_fp32"] = {k: v for k, v in mixed.items() if k not in ("D", "mu", "e_band", "n_e", "ranks")}
        out["forms"]["mixed_fp32"]["vs_fp64_batched"] = {
            "max_dD": float(np.abs(mixed["D"] - D_gpu).max()),
            "dE_band_per_atom": abs(mixed["e_band"] - eb_b) / s["n_atoms"], "dmu": abs(mixed["mu"] - mu_b)}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: the oracle's whole build of the same input ...")
        base, ref0, ref1 = oracle_builds(s, log)
        out["cpu_baseline"] = base
        out["accuracy"] = accuracy_vs_oracle(s, ref1, D_gpu, mu_b, eb_b, ne_b, ranks)
        log(f"[bench] accuracy: {out['accuracy']}")
        if mixed is not None:
            acc = accuracy_vs_oracle(s, ref1, mixed["D"], mixed["mu"], mixed["e_band"], mixed["n_e"], mixed["ranks"])
            acc["dN_e_bisection_fp64_weights"] = mixed["bisection_residual"]
            out["forms"]["mixed_fp32"]["accuracy"] = acc
            log(f"[bench] mixed form accuracy: {acc}")
    return out


def bisection_residual(plan, s, mu):
    """|g sum_i sum_mu f((eps - mu)/kT) w_mu - N_e| from every cluster's FP64 spectrum and weights at
    the build's mu (the electron count the bisection solves for; reading (ii) of the mixed form's
    electron-count target)."""
    g = float(s.get("spin_g", 2))
    tot = 0.0
    for i in range(s["n_atoms"]):
        e, w = plan.cluster_spectrum(i)
        tot += float(np.sum(0.5 * (1.0 - np.tanh(0.5 * (e - mu) / s["kT"])) * w))
    return abs(g * tot - s["n_electrons"])


if __name__ == "__main__":
    main()
